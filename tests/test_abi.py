"""Host-side checks of the GPU library that need no GPU: it loads, it exports
every symbol its headers declare, and its integer helpers (cell division,
Hilbert index) agree with the oracle and with plain arithmetic."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sba():
    import paper_2010_12548_amd as m
    m.lib()
    return m


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(sba_[a-z_0-9]+)\s*\(", txt))


@pytest.mark.parametrize("header", ["sba.h", "sba_debug.h"])
def test_exports_every_declared_symbol(sba, header):
    names = _declared(header)
    assert names, header
    L = sba.lib()
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in {header} but not exported"


def test_strerror_and_version(sba):
    L = sba.lib()
    assert L.sba_version().startswith(b"sba")
    for code in (0, -1, -2, -3, -4, -5):
        assert L.sba_strerror(code)
    assert L.sba_strerror(-99) == b"unknown error"


def test_build_rejects_bad_args_without_gpu(sba):
    import ctypes as C
    L = sba.lib()
    h = C.c_void_p(None)
    # null polygons and out-of-range eps are refused before any device call
    assert L.sba_build_approx(None, 64, None, None, C.byref(h)) == -1
    p = sba._Polys(0, None, None, None)
    assert L.sba_build_approx(C.byref(p), 1, None, None, C.byref(h)) == -1
    assert L.sba_build_approx(C.byref(p), (1 << 28) + 1, None, None, C.byref(h)) == -1
    assert L.sba_aggregate(None, None, 0, None, None, None, None) == -1


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 45, 70, 641, 707, 7071, 10606, 65535, 65537,
                               1 << 20, (1 << 20) + 1, 189812531, (1 << 28) - 1, 1 << 28])
def test_cell_division_exact(sba, s):
    rng = np.random.default_rng(s)
    top = (1 << 31) - 1
    n = np.concatenate([
        rng.integers(0, top, size=200000, dtype=np.int64),
        np.arange(0, 4096, dtype=np.int64),
        np.array([top, top - 1]),
        # multiples of s and their neighbours
        np.clip(np.arange(1, 3000, dtype=np.int64) * s + np.array([[-1], [0], [1]]), 0, top).ravel(),
        np.clip(top // s * s + np.arange(-3, 4), 0, top),
    ]).astype(np.uint32)
    q = sba.celldiv(s, n)
    np.testing.assert_array_equal(q.astype(np.int64), n.astype(np.int64) // s)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 16, 21])
def test_hilbert_matches_oracle(sba, orc, L):
    rng = np.random.default_rng(L)
    side = 1 << L
    pts = rng.integers(0, side, size=(3000, 2))
    for i, j in pts:
        d = sba.hilbert(L, i, j)
        assert d == orc.hilbert_d(L, int(i), int(j))
        assert sba.hilbert_cell(L, d) == (int(i), int(j))


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2010_12548_amd as m
    monkeypatch.setattr(m, "_LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(RuntimeError):
        m.lib()


def test_struct_layouts_match_header(sba, tmp_path):
    """The ctypes mirrors of the option and info structs have the sizes and
    field offsets the C compiler gives the header's structs."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"sba_build_opts": sba._Opts, "sba_info_t": sba._Info,
               "sba_pindex_opts": sba._PiOpts, "sba_pindex_info_t": sba._PiInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sba.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4, 5, 7, 8, 11, 12, 15, 16])
def test_hilbert_table_encoder_matches_oracle(sba, orc, L):
    """The probes' encoder that takes four levels at a time through a table
    gives the oracle's Hilbert index (every cell for small L, samples and
    the corners otherwise)."""
    lib = sba.lib()
    side = 1 << L
    if side <= 64:
        cells = [(i, j) for i in range(side) for j in range(side)]
    else:
        rng = np.random.default_rng(100 + L)
        cells = [tuple(map(int, c)) for c in rng.integers(0, side, size=(4000, 2))]
        cells += [(0, 0), (side - 1, 0), (0, side - 1), (side - 1, side - 1)]
    for i, j in cells:
        assert lib.sba_debug_hilbert_tab(L, i, j) == orc.hilbert_d(L, i, j), (L, i, j)

"""CPU-only checks of the C ABI: the library loads, exports every function that
include/gfq.h declares, and rejects bad arguments on the host before any GPU work."""
import ctypes
import os
import re

import pytest

from paper_0901_1413_amd import gfq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gfq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gfq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = gfq.load()
    names = declared_functions()
    assert "gfq_matmul" in names and "gfq_pack" in names and "gfq_matmul_batched" in names
    for name in names:
        assert hasattr(lib, name), name


def test_packed_bytes():
    assert gfq.packed_bytes(3, 10, 1) == 10 * 2 * 4 * 4
    assert gfq.packed_bytes(5, 3, 129) == 3 * 3 * 8 * 4
    assert gfq.packed_bytes(8, 3, 129) == 3 * 3 * 8 * 4
    assert gfq.packed_bytes(9, 3, 129) == 3 * 4 * 8 * 4
    assert gfq.packed_bytes(4, 0, 100) == 0
    assert gfq.packed_bytes(11, 3, 3) == 0
    assert gfq.packed_bytes(3, -1, 3) == 0


def test_host_validation_before_launch():
    lib = gfq.load()
    vp = ctypes.c_void_p
    assert lib.gfq_matmul(11, 4, 4, 4, vp(16), vp(16), vp(4096)) == -2
    assert lib.gfq_matmul(3, -1, 4, 4, vp(16), vp(16), vp(4096)) == -3
    assert lib.gfq_matmul(3, 4, 1 << 24, 4, vp(16), vp(16), vp(4096)) == -3
    assert lib.gfq_matmul(3, 4, 4, 4, vp(0), vp(16), vp(4096)) == -4
    assert lib.gfq_matmul(3, 4, 4, 4, vp(17), vp(16), vp(4096)) == -5
    assert lib.gfq_matmul(3, 4, 4, 4, vp(16), vp(64), vp(32)) == -6     # C overlaps A
    assert lib.gfq_matmul(3, 0, 4, 4, vp(0), vp(0), vp(0)) == 0         # empty: no-op
    assert lib.gfq_pack(3, 2, 2, vp(0), 2, vp(16)) == -4
    assert lib.gfq_pack(3, 2, 5, vp(1), 4, vp(16)) == -3                # ld < cols
    assert lib.gfq_unpack(6, 2, 2, vp(16), vp(0), 2) == -2
    assert lib.gfq_matmul_batched(-1, None) == -1
    assert lib.gfq_matmul_batched(0, None) == 0


def test_config_choice_and_checks():
    c = gfq.choose_config(3, 8192, 8192, 8192)
    assert c["k"] == 7 and c["rows"] in (256, 512, 1024, 2048) and c["split"] >= 1
    c5 = gfq.choose_config(5, 8192, 8192, 8192)
    assert 1 <= c5["k"] <= 10
    assert gfq.choose_config(3, 4, 3, 4)["k"] == 3        # k never exceeds l
    lib = gfq.load()
    bad = gfq.Config(11, 256, 1, 0)
    vp = ctypes.c_void_p
    assert lib.gfq_matmul_config(3, 4, 4, 4, vp(16), vp(4096), vp(8192), ctypes.byref(bad)) == -1
    bad = gfq.Config(8, 100, 1, 0)
    assert lib.gfq_matmul_config(3, 4, 4, 4, vp(16), vp(4096), vp(8192), ctypes.byref(bad)) == -1


def test_untuned_slab_width_keeps_tiles_filled():
    """Without a tuned entry the slab width is k = 7, except where k = 7 means 32-word
    (1024-column) tiles, i.e. three- and four-plane tables with 128-byte super-rows, and the
    product is at most 16 words (512 columns) wide: then k = 6 keeps 16-word tiles."""
    for q in (5, 7, 8, 9):
        assert gfq.choose_config(q, 1000, 1000, 512)["k"] == 6
        assert gfq.choose_config(q, 1000, 1000, 513)["k"] == 7       # 20 words
        assert gfq.choose_config(q, 1000, 1000, 4096)["k"] == 7
    for q in (3, 4):                                                   # k = 7: 256-byte rows
        assert gfq.choose_config(q, 1000, 1000, 200)["k"] == 7


def test_strerror():
    lib = gfq.load()
    for s in range(-10, 1):
        assert lib.gfq_strerror(s)


def test_choose_config_degenerate_shapes():
    """Empty products have no tiles; choosing their configuration must not divide by zero."""
    for q in (3, 4, 5, 7, 8, 9):
        for m, l, n in ((0, 4, 4), (4, 4, 0), (0, 0, 0), (5, 0, 7), (1, 1, 1)):
            c = gfq.choose_config(q, m, l, n)
            assert 1 <= c["k"] <= 10 and c["split"] >= 1


def test_tune_cache_text_roundtrip(tmp_path):
    """The tuning cache file is plain text; loading validates each entry (host logic only)."""
    f = tmp_path / "tune.txt"
    f.write_text("# arch mode q m_class l_class n_class k rows split variant\n"
                 "gfx950 0 3 13 13 13 7 2048 2\n"                # an entry without the variant column
                 "gfx950 1 5 9 10 0 6 256 1 0\n"
                 "gfx950 0 4 12 11 12 6 2048 1 1\n"              # GF(4) by Karatsuba
                 "gfx950 0 5 12 12 12 8 512 4 0 3000 2500\n"     # timed on a 3000 x . x 2500 product
                 "gfx950 2 5 13 13 13 3 0 0 0\n")                # Strassen-Winograd: 3 levels
    gfq.tune_clear()
    gfq.tune_load(str(f))
    out = tmp_path / "out.txt"
    gfq.tune_save(str(out))
    lines = [l.split() for l in out.read_text().splitlines() if not l.startswith("#")]
    # single-product lines gain the shape timed (absent: the class's largest, 2^class)
    assert sorted(lines) == sorted([["gfx950", "0", "3", "13", "13", "13", "7", "2048", "2", "0", "8192", "8192"],
                                    ["gfx950", "1", "5", "9", "10", "0", "6", "256", "1", "0"],
                                    ["gfx950", "0", "4", "12", "11", "12", "6", "2048", "1", "1", "4096", "4096"],
                                    ["gfx950", "0", "5", "12", "12", "12", "8", "512", "4", "0", "3000", "2500"],
                                    ["gfx950", "2", "5", "13", "13", "13", "3", "0", "0", "0"]])
    for bad_line in ("gfx950 0 3 13 13 13 11 2048 2\n",       # k = 11 is out of range
                     "gfx950 0 3 13 13 13 7 2048 2 1\n",      # no matrix route for F_3
                     "gfx950 0 4 13 13 13 7 2048 2 2\n",      # no such variant
                     "gfx950 0 3 13 13 13 7 2048 2 0 0 8192\n",      # a timed shape of 0 rows
                     "gfx950 0 3 13 13 13 7 2048 2 0 8192\n",        # half a shape
                     "gfx950 1 5 9 10 0 6 256 1 0 512 512\n",        # a shape on a batch entry
                     "gfx950 2 5 13 13 13 5 0 0 0\n",         # more levels than the maximum
                     "gfx950 0 3 13 13 13 7 0 2 0 8192 8192\n",      # a tile of 0 rows
                     "gfx950 0 3 13 13 13 7 -512 2 0 8192 8192\n",   # a negative tile height
                     "gfx950 0 5 13 13 13 7 768 2 0 8192 8192\n"):   # a height the API refuses
        gfq.tune_clear()
        bad = tmp_path / "bad.txt"
        bad.write_text(bad_line)
        with pytest.raises(gfq.GfqError):
            gfq.tune_load(str(bad))
        # a rejected entry leaves nothing in the cache
        left = tmp_path / "left.txt"
        gfq.tune_save(str(left))
        assert [l for l in left.read_text().splitlines() if not l.startswith("#")] == []
    gfq.tune_clear()
    out2 = tmp_path / "empty.txt"
    gfq.tune_save(str(out2))
    assert [l for l in out2.read_text().splitlines() if not l.startswith("#")] == []


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and says why, before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""

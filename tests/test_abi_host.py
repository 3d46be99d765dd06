"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/tsmm.h, validates arguments before
any HIP call, and derives plans from explicit device properties."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsmm.h")


@pytest.fixture(scope="module")
def T():
    from paper_2208_08088_amd import tsmm
    if not os.path.exists(tsmm.LIB_PATH):
        pytest.skip("libtsmm.so not built")
    tsmm._lib()
    return tsmm


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(tsmm_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tsmm_pack", "tsmm_plan", "tsmm_execute", "tsmm_plan_batched", "tsmm_execute_batched",
                     "tsmm_graph_create_batched", "tsmm_last_error", "tsmm_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(T):
    lib = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared entry point with a signature
    assert sorted(n for n, _, _ in T.SIGNATURES) == declared_functions()


def test_status_strings_and_version(T):
    lib = T._lib()
    for s in range(8):
        assert lib.tsmm_status_string(s)
    assert lib.tsmm_status_string(99) == b"unknown status"
    assert lib.tsmm_version() == 10100


def test_pack_validates_before_touching_hip(T):
    lib = T._lib()
    h = ctypes.c_void_p(0)
    assert lib.tsmm_pack(None, 4, 4, 0, 0, 0, None, None) == T.INVALID_VALUE
    assert lib.tsmm_pack(None, -1, 4, 0, 0, 0, None, ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_pack(None, 4, 4, 0, 0, 0, None, ctypes.byref(h)) == T.INVALID_VALUE  # NULL B
    assert b"B is NULL" in lib.tsmm_last_error()
    assert lib.tsmm_pack(ctypes.c_void_p(16), 4, 4, 7, 0, 0, None, ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_pack(ctypes.c_void_p(16), 4, 4, 0, 9, 0, None, ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_pack(ctypes.c_void_p(16), 4, 4, 0, 0, 5, None, ctypes.byref(h)) == T.INVALID_VALUE
    # split modes only for binary32 op N, and only within the fragment classes
    assert lib.tsmm_pack(ctypes.c_void_p(16), 4, 4, 0, T.F64, T.MODE_BF16X6, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    assert lib.tsmm_pack(ctypes.c_void_p(16), 4, 4, 1, T.F32, T.MODE_BF16X3, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    assert lib.tsmm_pack(ctypes.c_void_p(16), 300, 4, 0, T.F32, T.MODE_BF16X6, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    # empty operands need no device: a handle is returned
    assert lib.tsmm_pack(None, 0, 5, 0, T.F64, 0, None, ctypes.byref(h)) == T.SUCCESS and h.value
    nb = ctypes.c_size_t(1)
    assert lib.tsmm_packed_bytes(h, ctypes.byref(nb)) == T.SUCCESS and nb.value == 0
    lib.tsmm_packed_destroy(h)
    lib.tsmm_packed_destroy(None)
    lib.tsmm_plan_destroy(None)
    lib.tsmm_graph_destroy(None)


def test_pack_a_validates_before_touching_hip(T):
    lib = T._lib()
    h = ctypes.c_void_p(0)
    A = ctypes.c_void_p(16)
    assert lib.tsmm_pack_a(A, 4, 4, 4, T.F64, 0, 1.0, None, None) == T.INVALID_VALUE  # NULL out
    assert lib.tsmm_pack_a(A, -1, 4, 4, T.F64, 0, 1.0, None, ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_pack_a(None, 4, 4, 4, T.F64, 0, 1.0, None, ctypes.byref(h)) == T.INVALID_VALUE  # NULL A
    assert lib.tsmm_pack_a(A, 4, 4, 3, T.F64, 0, 1.0, None, ctypes.byref(h)) == T.INVALID_VALUE  # lda < k
    assert lib.tsmm_pack_a(A, 4, 4, 4, 9, 0, 1.0, None, ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_pack_a(A, 4, 4, 4, T.F32, 7, 1.0, None, ctypes.byref(h)) == T.INVALID_VALUE
    # bfloat16 A is read as it is; the split modes take binary32 with k <= 256
    assert lib.tsmm_pack_a(A, 4, 4, 4, T.BF16, 0, 1.0, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    assert lib.tsmm_pack_a(A, 4, 4, 4, T.F64, T.MODE_BF16X6, 1.0, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    assert lib.tsmm_pack_a(A, 4, 300, 300, T.F32, T.MODE_BF16X3, 1.0, None, ctypes.byref(h)) == T.NOT_SUPPORTED
    # an empty A needs no device; the handle is refused where a packed B goes
    assert lib.tsmm_pack_a(None, 0, 8, 8, T.F32, T.MODE_BF16X6, 2.0, None, ctypes.byref(h)) == T.SUCCESS
    assert h.value
    nb = ctypes.c_size_t(1)
    assert lib.tsmm_packed_bytes(h, ctypes.byref(nb)) == T.SUCCESS and nb.value == 0
    assert lib.tsmm_unpack(h, ctypes.c_void_p(16), None) == T.NOT_SUPPORTED
    assert lib.tsmm_packed_split_planes(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == T.NOT_SUPPORTED
    caps = T._Caps(256, 163840, 950)
    p = ctypes.c_void_p(0)
    assert lib.tsmm_plan_with_caps(0, 8, 8, 0, T.F32, ctypes.byref(caps), ctypes.byref(p)) == T.SUCCESS
    assert lib.tsmm_execute_packed_a(p, h, h, None, 0.0) != T.SUCCESS
    assert lib.tsmm_execute_packed_a(None, h, h, None, 0.0) == T.INVALID_VALUE
    lib.tsmm_plan_destroy(p)
    lib.tsmm_packed_destroy(h)


def test_plan_validation(T):
    lib = T._lib()
    h = ctypes.c_void_p(0)
    caps = T._Caps(256, 163840, 950)
    assert lib.tsmm_plan_with_caps(-1, 4, 4, 0, 0, ctypes.byref(caps), ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_plan_with_caps(4, 4, 4, 3, 0, ctypes.byref(caps), ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_plan_with_caps(4, 4, 4, 0, 5, ctypes.byref(caps), ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_plan_with_caps(4, 4, 4, 0, 0, None, ctypes.byref(h)) == T.INVALID_VALUE
    bad = T._Caps(0, 163840, 950)
    assert lib.tsmm_plan_with_caps(4, 4, 4, 0, 0, ctypes.byref(bad), ctypes.byref(h)) == T.INVALID_VALUE
    assert lib.tsmm_plan_with_caps(4, 4, 4, 0, 0, ctypes.byref(caps), None) == T.INVALID_VALUE
    # a caps-only plan cannot execute
    assert lib.tsmm_plan_with_caps(64, 8, 8, 0, 0, ctypes.byref(caps), ctypes.byref(h)) == T.SUCCESS
    assert lib.tsmm_execute(h, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1.0, 0.0) in (
        T.NO_DEVICE, T.SHAPE_MISMATCH)
    lib.tsmm_plan_destroy(h)


def test_plan_geometry_from_caps(T):
    # op N binary64, k = n = 8, m = 2^23: streaming kernel, k class 8, one
    # 16-column tile, vector mapping, grid capped at CUs * wg_per_cu
    p = T.plan_with_caps(1 << 23, 8, 8, "N")
    info = p.info()
    assert info["kernel"] == "stream" and info["kc"] == "8" and info["nt"] == "1" and info["vec"] == "1"
    tile = p.get_tile()
    grid = int(info["grid"].split("x")[0])
    assert grid == 256 * tile["wg_per_cu"]
    # odd k: scalar mapping
    assert T.plan_with_caps(1000, 16, 7, "N").info()["vec"] == "0"
    # tiny m: grid shrinks to the work
    assert int(T.plan_with_caps(16, 16, 16, "N").info()["grid"].split("x")[0]) == 1
    # beyond the fragment classes: the any-shape kernel
    assert T.plan_with_caps(100, 300, 16, "N").info()["kernel"] == "simple"
    # k beyond the classes: the k-slab kernel
    assert T.plan_with_caps(100, 16, 1000, "N").info()["kernel"] == "slab"


def test_plan_splitk_workspace(T):
    p = T.plan_with_caps(64, 64, 1 << 22, "T")
    info = p.info()
    assert info["kernel"] == "splitk"
    P = p.get_tile()["splitk"]
    assert 1 <= P <= 512
    assert p.workspace_bytes() == P * 64 * 64 * 8
    p.set_tile(kernel=T.KERNEL_SPLITK, splitk=100)
    assert p.workspace_bytes() == 100 * 64 * 64 * 8
    # output blocks: m = 100 > 64 -> two 64-row blocks, n = 20 -> 32-wide block
    q = T.plan_with_caps(100, 20, 4096, "T")
    grid = q.info()["grid"].split("x")
    assert int(grid[1]) == 2


def test_set_tile_validation(T):
    p = T.plan_with_caps(4096, 16, 16, "N")
    with pytest.raises(T.TsmmError) as e:
        p.set_tile(kernel=T.KERNEL_SPLITK)
    assert e.value.status == T.NOT_SUPPORTED
    with pytest.raises(T.TsmmError) as e:
        p.set_tile(kernel=T.KERNEL_STREAM, waves_per_wg=3)
    assert e.value.status == T.INVALID_VALUE
    with pytest.raises(T.TsmmError) as e:
        p.set_tile(kernel=T.KERNEL_STREAM, waves_per_wg=8)  # eight only for the wide kernels
    assert e.value.status == T.INVALID_VALUE
    with pytest.raises(T.TsmmError):
        p.set_tile(kernel=T.KERNEL_STREAM, rows_per_wave=16)  # no such instantiation
    p.set_tile(kernel=T.KERNEL_SIMPLE)
    assert p.info()["kernel"] == "simple"
    p.set_tile(kernel=T.KERNEL_STREAM, rows_per_wave=2, wg_per_cu=3)
    # 4096 rows = 256 tiles of 16 -> 128 wavefronts -> 32 workgroups of 4
    assert p.get_tile()["rows_per_wave"] == 2 and p.info()["grid"] == "32x1"
    big = T.plan_with_caps(1 << 22, 16, 16, "N")
    big.set_tile(kernel=T.KERNEL_STREAM, rows_per_wave=2, wg_per_cu=3)
    assert big.info()["grid"] == "768x1"


def test_set_mode_rules(T):
    p = T.plan_with_caps(4096, 64, 256, "N", dtype=__import__("torch").float32)
    p.set_mode("bf16x6")
    assert p.info()["kernel"] == "splitbf16" and p.info()["mode"] == "bf16x6"
    q = T.plan_with_caps(4096, 16, 16, "N")
    with pytest.raises(T.TsmmError) as e:
        q.set_mode("bf16x3")
    assert e.value.status == T.NOT_SUPPORTED


def test_tile_table_parsing(T, tmp_path):
    # a table is read once per process: check it in a child process
    import subprocess
    import sys
    key = T.table_key(950)
    tab = tmp_path / "t.txt"
    tab.write_text("# comment\n" + key + "N f64 native 8 1 2 : stream 2 4 6 1 1\n"
                   "T f64 native 4 4 2 : splitk 4 4 2 300 1\nB f32 native 0 0 0 : batched 0 8 1 1 1 2048\n")
    code = (
        "from paper_2208_08088_amd import tsmm as T\n"
        "p = T.plan_with_caps(1 << 23, 8, 8, 'N'); i = p.info(); t = p.get_tile()\n"
        "assert i['table'] == '1' and t['rows_per_wave'] == 2 and t['wg_per_cu'] == 6, (i, t)\n"
        "q = T.plan_with_caps(64, 64, 1 << 22, 'T'); assert q.get_tile()['splitk'] == 300 and q.info()['table'] == '1'\n"
        "r = T.plan_with_caps(1 << 23, 32, 32, 'N'); assert r.info()['table'] == '0'\n"
        "print('ok')\n")
    env = dict(os.environ, TSMM_TILE_TABLE=str(tab))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True)
    assert out.returncode == 0 and "ok" in out.stdout, out.stderr
    bad = tmp_path / "bad.txt"
    bad.write_text(key + "N f64 native 8 1 2 : nosuchkernel 2 4 6 1 1\n")
    code2 = ("from paper_2208_08088_amd import tsmm as T\n"
             "p = T.plan_with_caps(1 << 23, 8, 8, 'N'); assert p.info()['table'] == '0'\n"
             "print('ok')\n")
    out = subprocess.run([sys.executable, "-c", code2], cwd=ROOT, env=dict(os.environ, TSMM_TILE_TABLE=str(bad)),
                         capture_output=True, text=True)
    assert out.returncode == 0 and "ok" in out.stdout, out.stderr
    out = subprocess.run([sys.executable, "-c", code2], cwd=ROOT,
                         env=dict(os.environ, TSMM_TILE_TABLE=str(bad), TSMM_STRICT_TABLE="1"),
                         capture_output=True, text=True)
    assert out.returncode != 0 and "tile table" in out.stderr
    # a batched entry needs the chunk field and the batched kernel, and only
    # the batched layout takes that kernel
    for line in ("B f32 native 0 0 0 : batched 0 8 1 1 1\n", "B f32 native 0 0 0 : stream 0 8 1 1 1 2048\n",
                 "N f64 native 8 1 2 : batched 2 4 6 1 1\n"):
        bad.write_text(key + "N f64 native 8 1 2 : stream 2 4 6 1 1\n" + line)
        out = subprocess.run([sys.executable, "-c", code2], cwd=ROOT, env=dict(os.environ, TSMM_TILE_TABLE=str(bad)),
                             capture_output=True, text=True)
        assert out.returncode == 0 and "ok" in out.stdout, (line, out.stderr)


def test_tile_table_keys(T, tmp_path):
    # a table is used only where its key lines (architecture, HIP runtime,
    # library version) match; otherwise the plan takes built-in tiles, or
    # fails with TSMM_ERROR_TABLE under TSMM_STRICT_TABLE
    import subprocess
    import sys
    key = T.table_key(950)
    lines = dict(l.split()[1:] for l in key.splitlines())
    assert lines["arch"] == "gfx950" and int(lines["libtsmm"]) == T.version() and int(lines["hip"]) > 0
    with pytest.raises(T.TsmmError):
        T.table_key(-1)
    entry = "N f64 native 8 1 2 : stream 2 4 6 1 1\n"
    probe = ("from paper_2208_08088_amd import tsmm as T\n"
             "p = T.plan_with_caps(1 << 23, 8, 8, 'N', gcn_arch=%d); print('table=' + p.info()['table'])\n")

    def run(text, arch=950, strict=False):
        tab = tmp_path / "k.txt"
        tab.write_text(text)
        env = dict(os.environ, TSMM_TILE_TABLE=str(tab), TSMM_LOG="1")
        if strict:
            env["TSMM_STRICT_TABLE"] = "1"
        return subprocess.run([sys.executable, "-c", probe % arch], cwd=ROOT, env=env, capture_output=True,
                              text=True)

    out = run(key + entry)
    assert out.returncode == 0 and "table=1" in out.stdout, out.stderr
    foreign = {
        "another architecture": (key.replace("gfx950", "gfx942"), "is for gfx942"),
        "another library version": (key.replace("libtsmm %d" % T.version(), "libtsmm 10000"), "libtsmm 10000"),
        "another HIP runtime": (key.replace("hip %s" % lines["hip"], "hip 60000000"), "HIP runtime 60000000"),
        "no key lines": ("", "no key lines"),
    }
    for what, (k, why) in foreign.items():
        out = run(k + entry)
        assert out.returncode == 0 and "table=0" in out.stdout, (what, out.stderr)
        assert "tile table" in out.stderr and why in out.stderr, (what, out.stderr)  # the fallback is logged
        out = run(k + entry, strict=True)
        assert out.returncode != 0 and "tile table" in out.stderr and why in out.stderr, (what, out.stderr)
    # the keyed architecture only: a plan for another device takes built-in tiles
    out = run(key + entry, arch=942)
    assert out.returncode == 0 and "table=0" in out.stdout, out.stderr
    out = run("key arch gfx950\nkey hip\n" + entry, strict=True)
    assert out.returncode != 0 and "malformed key line" in out.stderr


def test_shipped_tile_table_is_keyed_for_this_library(T):
    # the install-time table in the package carries this library's version
    path = os.path.join(ROOT, "paper_2208_08088_amd", "tile_table.txt")
    keys = [l.split()[1:] for l in open(path) if l.startswith("key ")]
    assert dict(keys)["libtsmm"] == str(T.version()) and dict(keys)["arch"] == "gfx950"


def test_valu64_tile_rules(T):
    p = T.plan_with_caps(1 << 20, 128, 128, "N")
    p.set_tile(kernel=T.KERNEL_VALU64, rows_per_wave=32, waves_per_wg=4, wg_per_cu=2)
    info = p.info()
    # 128 columns / 32 per wavefront = 4 column groups = one group of 4 wavefronts
    assert info["kernel"] == "valu64" and info["grid"] == "512x1"
    with pytest.raises(T.TsmmError):  # n not a multiple of the column block
        T.plan_with_caps(1000, 40, 128, "N").set_tile(kernel=T.KERNEL_VALU64, rows_per_wave=32)
    with pytest.raises(T.TsmmError):  # k not a multiple of 8
        T.plan_with_caps(1000, 32, 12, "N").set_tile(kernel=T.KERNEL_VALU64, rows_per_wave=16)
    with pytest.raises(T.TsmmError):  # binary32 is not served by it
        T.plan_with_caps(1000, 32, 32, "N", dtype=__import__("torch").float32).set_tile(kernel=T.KERNEL_VALU64)
    q = T.plan_with_caps(1000, 256, 64, "N")
    q.set_tile(kernel=T.KERNEL_VALU64, rows_per_wave=16)
    assert q.info()["grid"].endswith("x4")


def test_wide_tile_rules(T):
    f32 = __import__("torch").float32
    # n = 256: two 32-row tiles per wavefront, 256 rows per workgroup, one
    # workgroup per compute unit
    p = T.plan_with_caps(1 << 24, 256, 256, "N", dtype=f32)
    p.set_tile(kernel=T.KERNEL_WIDE)
    t, info = p.get_tile(), p.info()
    assert info["kernel"] == "wide" and t["rows_per_wave"] == 2 and t["wg_per_cu"] == 1
    assert info["grid"] == "256x1" and info["kc"] == "256" and info["nt"] == "8"
    for mode in ("bf16x3", "bf16x6"):
        q = T.plan_with_caps(1000, 256, 256, "N", dtype=f32).set_mode(mode)
        q.set_tile(kernel=T.KERNEL_WIDE)
        assert q.info()["grid"] == "4x1"  # 1000 rows -> 4 workgroup tiles of 256
    # n = 128: four 32-row tiles, k = 40 -> packed k class 64
    r = T.plan_with_caps(70001, 128, 40, "N", dtype=f32)
    r.set_tile(kernel=T.KERNEL_WIDE)
    assert r.get_tile()["rows_per_wave"] == 4 and r.info()["kc"] == "64" and r.info()["grid"] == "137x1"
    r.set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=2)
    assert r.info()["grid"] == "256x1"
    r.set_mode("bf16x6")  # split modes: two 32-row tiles only
    r.set_tile(kernel=T.KERNEL_WIDE)
    assert r.get_tile()["rows_per_wave"] == 2
    with pytest.raises(T.TsmmError):
        r.set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=4)
    # eight wavefronts (two per SIMD) with one 32-row tile each: 256 rows
    # per workgroup again
    for mode in ("native", "bf16x3", "bf16x6"):
        w = T.plan_with_caps(1 << 24, 256, 256, "N", dtype=f32)
        if mode != "native":
            w.set_mode(mode)
        w.set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=1, waves_per_wg=8)
        assert w.info()["waves"] == "8" and w.info()["block"] == "512" and w.info()["grid"] == "256x1"
        w = T.plan_with_caps(1000, 128, 64, "N", dtype=f32).set_mode(mode) if mode != "native" else \
            T.plan_with_caps(1000, 128, 64, "N", dtype=f32)
        w.set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=1, waves_per_wg=8)
        assert w.info()["grid"] == "4x1"
    bad = [
        (dict(m=1000, n=192, k=256, dtype=f32), {}),                     # n not 128 / 256
        (dict(m=1000, n=256, k=100, dtype=f32), {}),                     # k % 8 != 0
        (dict(m=1000, n=256, k=512, dtype=f32), {}),                     # k > 256
        (dict(m=1000, n=256, k=256, dtype=__import__("torch").float64), {}),  # binary64
        (dict(m=1000, n=256, k=256, dtype=f32), dict(rows_per_wave=4)),  # 512 accumulators
        (dict(m=1000, n=256, k=256, dtype=f32), dict(wg_per_cu=2)),
        (dict(m=1000, n=256, k=256, dtype=f32), dict(nsplit=2)),
        (dict(m=1000, n=256, k=256, dtype=f32), dict(rows_per_wave=2, waves_per_wg=8)),  # 256 registers
        (dict(m=1000, n=256, k=256, dtype=f32), dict(rows_per_wave=1, waves_per_wg=4)),  # not built
        (dict(m=1000, n=256, k=256, dtype=f32), dict(waves_per_wg=2)),
    ]
    for shape, extra in bad:
        with pytest.raises(T.TsmmError):
            T.plan_with_caps(shape["m"], shape["n"], shape["k"], "N", dtype=shape["dtype"]).set_tile(
                kernel=T.KERNEL_WIDE, **extra)
    # op T never
    with pytest.raises(T.TsmmError):
        T.plan_with_caps(256, 256, 4096, "T", dtype=f32).set_tile(kernel=T.KERNEL_WIDE)


def test_slab_tile_rules(T):
    torch = __import__("torch")
    # the paper's workload: square A (25600 x 25600) times B 25600 x 240.
    # binary64: 1 row tile per wavefront (16 tiles x 8 accumulator
    # registers), 64-row blocks -> 400 blocks; 3 parts of k fill 1200 of
    # 1280 workgroup slots (the fewest parts that fill 90%)
    p = T.plan_with_caps(25600, 240, 25600, "N")
    assert p.info()["kernel"] == "slab"
    p.set_tile(kernel=T.KERNEL_SLAB)  # the built-in default, whatever the tile table holds
    t, info = p.get_tile(), p.info()
    assert t["rows_per_wave"] == 1 and t["splitk"] == 3
    assert info["kc"] == "25600" and info["nt"] == "16" and info["grid"] == "256x1"
    assert p.workspace_bytes() == 3 * 1600 * 16 * 64 * 4 * 8
    # binary32: 2 row tiles (128-row blocks -> 200), 5 parts
    q = T.plan_with_caps(25600, 240, 25600, "N", dtype=torch.float32)
    q.set_tile(kernel=T.KERNEL_SLAB)
    assert q.info()["kernel"] == "slab" and q.get_tile()["rows_per_wave"] == 2 and q.get_tile()["splitk"] == 5
    # enough row blocks: no split, no workspace
    r = T.plan_with_caps(1 << 22, 64, 1000, "N")
    assert r.info()["kernel"] == "slab" and r.get_tile()["splitk"] == 1 and r.workspace_bytes() == 0
    assert r.info()["kc"] == "1024"  # 1000 rounded up to whole 32-k slabs
    r.set_tile(kernel=T.KERNEL_SLAB, splitk=3)
    assert r.workspace_bytes() == 3 * (1 << 18) * 4 * 64 * 4 * 8
    # k within the streaming classes: streaming by default, slab on request
    s = T.plan_with_caps(100000, 64, 128, "N")
    assert s.info()["kernel"] == "stream"
    s.set_tile(kernel=T.KERNEL_SLAB)
    assert s.info()["kernel"] == "slab" and s.info()["kc"] == "128"
    bad = [
        (dict(m=1000, n=64, k=1000), dict(splitk=33)),          # more parts than 32-k slabs
        (dict(m=1000, n=64, k=1000), dict(wg_per_cu=2)),
        (dict(m=1000, n=64, k=1000), dict(nsplit=2)),
        (dict(m=1000, n=256, k=1000), dict(rows_per_wave=4)),   # 512 accumulator registers: no instantiation
        (dict(m=1000, n=64, k=16), {}),                         # k class 16: not whole slabs
    ]
    for shape, extra in bad:
        with pytest.raises(T.TsmmError):
            T.plan_with_caps(shape["m"], shape["n"], shape["k"], "N").set_tile(kernel=T.KERNEL_SLAB, **extra)
    # k past 2^20: the any-shape kernel
    assert T.plan_with_caps(1000, 16, 1000, "N", dtype=torch.float32).info()["kernel"] == "slab"
    assert T.plan_with_caps(100, 64, (1 << 20) + 32, "N").info()["kernel"] == "simple"
    with pytest.raises(T.TsmmError):
        T.plan_with_caps(1000, 64, 1000, "N", dtype=torch.bfloat16).set_tile(kernel=T.KERNEL_SLAB)


def test_tune_validates_before_any_hip_call(T):
    lib = T._lib()
    p = T.plan_with_caps(4096, 16, 16, "N")
    # NULL packed operand / C
    assert lib.tsmm_plan_tune(p.handle, None, None, None, 3, None) == T.INVALID_VALUE
    assert lib.tsmm_plan_tune(None, None, None, None, 3, None) == T.INVALID_VALUE
    lib.tsmm_tune_cache_clear()  # no-op without entries


def test_colmajor_plan_rules(T):
    torch = __import__("torch")
    # binary64, m a multiple of 2: the column-major kernel; 32 m indices per
    # wavefront block, 4 wavefronts per workgroup
    p = T.plan_with_caps(1 << 20, 64, 64, "C")
    info = p.info()
    assert info["kernel"] == "colmajor" and info["op"] == "C"
    assert p.get_tile()["nsplit"] == 1
    # n = 256 at k class 256: at most 4 column tiles per group -> 4 groups
    q = T.plan_with_caps(1 << 20, 256, 256, "C")
    assert q.info()["kernel"] == "colmajor" and q.get_tile()["nsplit"] == 4
    # odd m (binary64) or m not a multiple of 4 (binary32): any-shape kernel
    assert T.plan_with_caps(1001, 16, 16, "C").info()["kernel"] == "simple"
    assert T.plan_with_caps(1002, 16, 16, "C", dtype=torch.float32).info()["kernel"] == "simple"
    assert T.plan_with_caps(1004, 16, 16, "C", dtype=torch.float32).info()["kernel"] == "colmajor"
    # k beyond 256: any-shape kernel
    assert T.plan_with_caps(1000, 16, 300, "C").info()["kernel"] == "simple"
    with pytest.raises(T.TsmmError):
        T.plan_with_caps(1 << 20, 64, 64, "C").set_tile(kernel=T.KERNEL_COLMAJOR, waves_per_wg=2)
    with pytest.raises(T.TsmmError):
        T.plan_with_caps(1 << 20, 64, 64, "C").set_tile(kernel=T.KERNEL_STREAM)
    with pytest.raises(T.TsmmError) as e:
        T.plan_with_caps(1000, 16, 16, "C", dtype=torch.bfloat16)
    assert e.value.status == T.NOT_SUPPORTED

"""Host checks of the install-time autotuner (no GPU): every shape class
yields candidate tiles the planner accepts, every kernel a candidate can
name has a tile-table name, and the table key it writes is the one
tsmm_plan looks up (the plan reports table=1 for it)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_2208_08088_amd import tsmm
    if not os.path.exists(tsmm.LIB_PATH):
        pytest.skip("libtsmm.so not built")
    from paper_2208_08088_amd import autotune
    return autotune


def test_every_class_has_valid_candidates(A):
    T = A.T
    for name, (layout, dt, mode, m, n, k) in A.CLASSES.items():
        if layout == "B":
            continue  # batched plans need a device
        p = T.plan_with_caps(m, n, k, layout, dtype=dt)
        if mode != "native":
            p.set_mode(mode)
        valid = []
        for cand in A.candidates(p):
            try:
                p.set_tile(**cand)
            except T.TsmmError:
                continue
            valid.append(p.get_tile())
        assert valid, name
        for t in valid:
            assert t["kernel"] in A._KERNEL_NAME, (name, t)


def test_written_keys_are_the_planner_keys(A, tmp_path):
    # one entry per class as the autotuner formats it; a child process
    # (the table is read once per process) plans each class from it
    lines = []
    for name, (layout, dt, mode, m, n, k) in A.CLASSES.items():
        if layout == "B":
            continue
        p = A.T.plan_with_caps(m, n, k, layout, dtype=dt)
        if mode != "native":
            p.set_mode(mode)
        t = p.get_tile()
        kc, nt, mcl = A.table_key(layout, dt, mode, m, n, k)
        lines.append("%s %s %s %d %d %d : %s %d %d %d %d %d" % (
            layout, A._DT_NAME[dt], mode, kc, nt, mcl, A._KERNEL_NAME[t["kernel"]], t["rows_per_wave"],
            t["waves_per_wg"], t["wg_per_cu"], t["splitk"], t["nsplit"]))
    tab = tmp_path / "t.txt"
    tab.write_text(A.T.table_key(950) + "\n".join(lines) + "\n")
    code = ("import torch\n"
            "from paper_2208_08088_amd import autotune as A\n"
            "for name, (layout, dt, mode, m, n, k) in A.CLASSES.items():\n"
            "    if layout == 'B': continue\n"
            "    p = A.T.plan_with_caps(m, n, k, layout, dtype=dt)\n"
            "    if mode != 'native': p.set_mode(mode)\n"
            "    assert p.info()['table'] == '1', (name, p.describe())\n"
            "print('ok')\n")
    env = dict(os.environ, TSMM_TILE_TABLE=str(tab), TSMM_STRICT_TABLE="1")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True)
    assert out.returncode == 0 and "ok" in out.stdout, out.stderr[-2000:]


def test_ties_go_to_the_tile_that_reads_A_least(A):
    from paper_2208_08088_amd import tsmm as T
    t = lambda w, kern=T.KERNEL_STREAM, ns=2: dict(kernel=kern, rows_per_wave=1, waves_per_wg=4, wg_per_cu=w,
                                                   splitk=1, nsplit=ns)
    # streaming kernel with column groups: the fewest resident workgroups
    ms, tile = A.pick([(5.00, t(4)), (5.05, t(1)), (5.02, t(2))])
    assert tile["wg_per_cu"] == 1 and ms == 5.05
    # outside TIE the fastest stays
    ms, tile = A.pick([(5.00, t(4)), (5.00 * (1 + A.TIE) + 0.01, t(1))])
    assert tile["wg_per_cu"] == 4
    # equal counts: the faster one
    ms, tile = A.pick([(5.01, t(2)), (5.00, t(2)), (4.99 * (1 + 2 * A.TIE), t(8))])
    assert ms == 5.00
    # column-major kernel with column groups: the most resident workgroups
    C = T.KERNEL_COLMAJOR
    ms, tile = A.pick([(5.00, t(1, C)), (5.05, t(16, C)), (5.02, t(4, C))])
    assert tile["wg_per_cu"] == 16
    # no column groups: the fastest
    ms, tile = A.pick([(5.02, t(1, ns=1)), (5.00, t(8, ns=1))])
    assert tile["wg_per_cu"] == 8
    # streaming kernel: then the fewest row tiles per wavefront
    r = lambda rt: dict(t(1), rows_per_wave=rt)
    ms, tile = A.pick([(5.00, r(2)), (5.01, r(1))])
    assert tile["rows_per_wave"] == 1
    # one column group before column groups, for either kernel
    for kern in (T.KERNEL_STREAM, C):
        ms, tile = A.pick([(5.00, t(1, kern)), (5.00, t(16, kern)), (5.05, t(2, kern, ns=1))])
        assert tile["nsplit"] == 1

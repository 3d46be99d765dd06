"""Build libtsmm.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2208_08088_amd.build [--force] [-j N]

Every translation unit is compiled with hipcc for gfx950 only, then linked
into ``paper_2208_08088_amd/libtsmm.so``.  Objects live in
``paper_2208_08088_amd/_build/`` and are rebuilt when a source or header is
newer, or always with ``--force``.  The benchmark's bandwidth-ceiling
kernels (``ceiling/k_ceiling.hip``) are built the same way into
``paper_2208_08088_amd/libtsmm_ceiling.so``, a library of their own.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtsmm.so")
CEIL_SRC = os.path.join(HERE, "ceiling", "k_ceiling.hip")
CEIL_LIB = os.path.join(HERE, "libtsmm_ceiling.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable",
          # packed fp32 vector instructions are disabled for all device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC]


# Per-file extra flags (none at present: the architectural-register form of
# the matrix-core products, -mllvm -amdgpu-mfma-vgpr-form, was measured 18%
# slower on the binary64 streaming kernels and does not build the bfloat16
# ones; only the ceiling loop takes it).
EXTRA = {}


def flags_of(src):
    return CFLAGS + EXTRA.get(os.path.basename(src), [])


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers_mtime():
    hs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return max(os.path.getmtime(h) for h in hs)


def _obj(src):
    # the object name carries a digest of its flags, so a flag change rebuilds it
    import hashlib
    tag = hashlib.sha256(" ".join(flags_of(src)).encode()).hexdigest()[:8]
    return os.path.join(BUILD, "%s.%s.o" % (os.path.basename(src), tag))


def _compile(src):
    obj = _obj(src)
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *flags_of(src), "-c", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (os.path.basename(src), out))
    os.replace(tmp, obj)
    return src, out


def build(force: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hmt = _headers_mtime()
    todo = []
    for src in sources():
        obj = _obj(src)
        if force or not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(src), hmt):
            todo.append(src)
    jobs = jobs or min(8, os.cpu_count() or 1)
    if todo:
        # biggest translation units first
        todo.sort(key=lambda s: -os.path.getsize(s))
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, out in ex.map(_compile, todo):
                if verbose:
                    print("[build] compiled %s" % os.path.basename(src), flush=True)
                if out.strip() and verbose:
                    print(out, flush=True)
    objs = [_obj(s) for s in sources()]
    if force or todo or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
        os.replace(tmp, LIB)
        if verbose:
            print("[build] linked %s" % LIB, flush=True)
    build_ceiling(force)
    return LIB


def build_ceiling(force: bool = False) -> str:
    """The benchmark's bandwidth-ceiling kernels, a library of their own."""
    if force or not os.path.exists(CEIL_LIB) or os.path.getmtime(CEIL_LIB) < os.path.getmtime(CEIL_SRC):
        tmp = CEIL_LIB + ".tmp%d" % os.getpid()
        # matrix-core products write their architectural-register form, so the
        # ceiling loop carries its accumulators without copies
        r = subprocess.run([HIPCC, *CFLAGS, "-mllvm", "-amdgpu-mfma-vgpr-form", "-shared", CEIL_SRC, "-o", tmp],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for k_ceiling.hip:\n%s" % (r.stdout + r.stderr))
        os.replace(tmp, CEIL_LIB)
    return CEIL_LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args(argv)
    build(force=a.force, jobs=a.j)


if __name__ == "__main__":
    sys.exit(main())

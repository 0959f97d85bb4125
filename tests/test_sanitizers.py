"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host-side sources (kernel-set builder, row-kernel table image, Marching Cubes case tables,
  sweep constants) are built with g++ and both sanitizers into a small driver, ``sanitize/host_checks.cpp``,
  and run.
* The C oracle is built with gcc and both sanitizers into a shared library, loaded by a child Python with the
  sanitizer runtime preloaded, and drives scans (tiny grids, every binning and both metrics, a deskewed
  sweep) through it.
Any report aborts the child (``-fno-sanitize-recover=all``) and fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_20081_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                                reason="needs g++ and the ROCm headers")


def _run(cmd, **kw):
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert out.returncode == 0, (" ".join(cmd), out.stdout[-3000:], out.stderr[-3000:])
    return out


def test_library_host_code_under_sanitizers(tmp_path):
    objs = []
    for src in ("kernel_set.cpp", "mesh.cpp", "deskew.cpp"):
        obj = str(tmp_path / (src + ".o"))
        _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
              *SAN, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_checks")
    _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
          *SAN, os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), *objs, "-o", exe])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert out.stdout.startswith("ok")


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", *SAN,
          os.path.join(ROOT, "oracle", "dbtsdf_oracle.c"), "-o", lib, "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    code = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
from oracle import oracle as O
O._LIB_PATH = %r
for kw in (dict(kernel_size=5, binning="cube26", shadow_r2=4, hit_threshold=2, hit_max=3),
           dict(kernel_size=7, binning="azel", bins_az=8, bins_el=5, shadow_r2=6, metric="l1"),
           dict(kernel_size=11, binning="cube26", shadow_r2=9, shadow_model="cone", cone_deg=35.0, dedup=False)):
    o = O.Oracle((24, 22, 20), 0.1, (0.0, 0.0, 0.0), **kw)
    m, p = o.new_grid()
    rng = np.random.default_rng(1)
    pose = np.eye(4, dtype=np.float32)
    pose[:3, 3] = (1.2, 1.1, 1.0)
    for _ in range(3):
        pts = rng.uniform(-1.2, 1.2, (400, 3)).astype(np.float32)
        pts[::37] = np.nan
        o.integrate(m, p, pose, pts, count_traffic=True)
    end = pose.copy()
    end[:3, 3] += 0.1
    o.integrate_deskew(m, p, pose, end, pts, np.linspace(-0.1, 1.1, len(pts)).astype(np.float32), "yaw")
    o.read_distance(m, p)
print("ok")
""" % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=" ".join(x for x in (asan, ubsan) if os.path.isabs(x)),
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1")
    out = _run([sys.executable, "-c", code], env=env)
    assert out.stdout.strip().endswith("ok")

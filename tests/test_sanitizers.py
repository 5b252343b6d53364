"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C loops, driven by tests/native/oracle_sanitize.c on small
  seeded inputs whose buffers end exactly at their last entry, with
  cross-checks between independent oracle functions.
* The library's host side (argument validation, method and working-memory
  planning, the autotuning table's JSON reader and writer), driven by
  tests/native/abi_sanitize.c through the C ABI: the host code is compiled
  with the sanitizers (the device code is not: GPU sanitizers are not used),
  and no call reaches a GPU.
"""
import os
import shutil
import subprocess
import concurrent.futures

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1705_08743_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

# host-only sanitizer flags for hipcc: each one behind -Xarch_host, so that
# no device code is built with them
HOST_SAN = []
for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"):
    HOST_SAN += ["-Xarch_host", flag]


def _run(cmd, **kw):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert res.returncode == 0, "%s\n%s" % (" ".join(cmd), res.stdout[-4000:])
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(NATIVE, "oracle_sanitize.c"),
          "-o", exe])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "ok" in out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="hipcc / ROCm clang not found")
def test_host_abi_under_sanitizers(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC] + HOST_SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + common + ["-c", src, "-o", obj])
        return obj

    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libsemiring_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", lib] + objs)
    exe = str(tmp_path / "abi_san")
    _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), os.path.join(NATIVE, "abi_sanitize.c"),
          "-L", str(tmp_path), "-lsemiring_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", HIP_VISIBLE_DEVICES="")
    env.pop("SR_AUTOTUNE_FILE", None)
    out = _run([exe, str(scratch)], env=env)
    assert "ok" in out

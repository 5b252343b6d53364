"""Build libsemiring.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Each source is compiled to a position-independent object in parallel (in
``_build/`` next to this file), then the objects are linked into the shared
library, which replaces the old one atomically."""
import concurrent.futures
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsemiring.so")
OBJ_DIR = os.path.join(PKG, "_build")
ARCH = "gfx950"
# packed FP32 instructions stay off in every device pass
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _filtered(text):
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())


def _jobs():
    env = os.environ.get("MAX_JOBS", "")
    n = int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def build(verbose: bool = False, extra_flags=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    tag = "%d" % os.getpid()
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + "." + tag + ".o")
        cmd = [hipcc] + FLAGS + list(extra_flags) + ["-c", src, "-o", obj]
        res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return src, obj, cmd, res.returncode, _filtered(res.stdout)

    with concurrent.futures.ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, srcs))
    objs = []
    for src, obj, cmd, rc, out in results:
        if verbose:
            print(" ".join(cmd), flush=True)
            if out:
                print(out)
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, out))
        objs.append(obj)
    tmp = LIB + ".tmp" + tag
    cmd = [hipcc, "--offload-arch=" + ARCH, "-fPIC", "-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + _filtered(res.stdout))
    os.replace(tmp, LIB)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(INCLUDE, "semiring.h")]
    return any(os.path.getmtime(p) > t for p in deps)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    sys.exit(0)

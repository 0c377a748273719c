"""Builds libpct's HIP sources for the CPU with AddressSanitizer, against the
stand-in runtime in this folder (hip/hip_runtime.h, emu_runtime.cpp).

The kernel sources are compiled unchanged except for one textual rewrite:
a dynamic LDS declaration `extern __shared__ T name[];` becomes a pointer to
the launch's LDS buffer.  The result is `_build/libpct_emu.so`, rebuilt when
any input changes.  Run as `python tests/emu/build_emu.py`."""
import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2403_07631_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libpct_emu.so")
CXX = os.environ.get("CXX", "g++")
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-fsanitize=address",
         "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-Wno-unused-variable", "-Wno-unused-function",
         "-DPCT_EMU=1", "-U_FORTIFY_SOURCE", "-D_FORTIFY_SOURCE=0"]

DYN_SHARED = re.compile(r"extern\s+__shared__\s+(\w+)\s+(\w+)\s*\[\s*\]\s*;")


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in hip]


def inputs():
    headers = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    files = sources() + headers + [os.path.join(ROOT, "include", "pct.h"),
                         os.path.join(HERE, "hip", "hip_runtime.h"), os.path.join(HERE, "emu_runtime.cpp"),
                         os.path.abspath(__file__)]
    return files


def digest():
    h = hashlib.sha256()
    for f in inputs():
        h.update(f.encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()


def _balanced(text, i):
    """Index just past the parenthesis that closes the one at text[i]."""
    depth = 0
    for j in range(i, len(text)):
        if text[j] == "(":
            depth += 1
        elif text[j] == ")":
            depth -= 1
            if depth == 0:
                return j + 1
    raise ValueError("unbalanced parentheses")


def rewrite(src):
    """Dynamic LDS declarations become pointers to the launch's LDS buffer;
    every kernel with __launch_bounds__(B) checks at entry that the launch
    has at most B threads per workgroup."""
    text = DYN_SHARED.sub(lambda m: f"{m.group(1)}* {m.group(2)} = ({m.group(1)}*)::emu::dyn_smem();",
                          open(src).read())
    out, pos = [], 0
    key = "__launch_bounds__("
    while True:
        i = text.find(key, pos)
        if i < 0:
            out.append(text[pos:])
            break
        e = _balanced(text, i + len(key) - 1)
        expr = text[i + len(key):e - 1]
        depth = 0
        for k, ch in enumerate(expr):    # the first argument: threads per workgroup
            depth += ch == "("
            depth -= ch == ")"
            if ch == "," and depth == 0:
                expr = expr[:k]
                break
        body = text.find("{", e)
        out.append(text[pos:body + 1])
        out.append(f" ::emu::check_launch_bound((int)({expr}), __func__);")
        pos = body + 1
    return "".join(out)


def build(force=False):
    os.makedirs(OUT, exist_ok=True)
    stamp = os.path.join(OUT, "digest")
    d = digest()
    if not force and os.path.exists(LIB) and os.path.exists(stamp) and open(stamp).read() == d:
        return LIB
    jobs = []
    for src in sources():
        cpp = os.path.join(OUT, os.path.basename(src)[:-4] + ".cpp")
        with open(cpp, "w") as fh:
            fh.write(f'#line 1 "{src}"\n' + rewrite(src))
        jobs.append(cpp)
    jobs.append(os.path.join(HERE, "emu_runtime.cpp"))
    inc = ["-I", HERE, "-I", CSRC, "-I", os.path.join(ROOT, "include")]

    def compile_one(cpp):
        obj = os.path.join(OUT, os.path.basename(cpp)[:-4] + ".o")
        r = subprocess.run([CXX, *FLAGS, *inc, "-c", cpp, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {cpp} failed:\n{r.stderr[-6000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, jobs))
    r = subprocess.run([CXX, *FLAGS, "-shared", *objs, "-o", LIB], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking {LIB} failed:\n{r.stderr[-4000:]}")
    with open(stamp, "w") as fh:
        fh.write(d)
    return LIB


def asan_runtime():
    """Path of the AddressSanitizer runtime that must be preloaded into a
    Python process that loads the library."""
    r = subprocess.run([CXX, "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))

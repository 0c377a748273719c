"""libpct's HIP kernels built for the CPU with AddressSanitizer (tests/emu) and
run on the same seeded cases as the GPU parity tests, against the oracle.

This checks the kernel sources themselves without a GPU: indexing (every
global and LDS access is bounds-checked by the sanitizer), barrier placement
(wavefronts are resumed in order, reversed and shuffled) and the arithmetic
(results must equal the oracle's exactly where the GPU tests require it).
Each group of cases runs in a child process with the sanitizer preloaded."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
sys.path.insert(0, EMU)

import build_emu  # noqa: E402


@pytest.fixture(scope="module")
def emu_lib():
    try:
        build_emu.asan_runtime()
    except Exception as e:  # pragma: no cover - toolchain without ASan
        pytest.skip(f"no AddressSanitizer runtime: {e}")
    return build_emu.build()


def _env(order):
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_emu.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["EMU_ORDER"] = order
    env["OMP_NUM_THREADS"] = "1"
    return env


def _start(cases, order):
    return subprocess.Popen([sys.executable, os.path.join(EMU, "driver.py"), *cases], env=_env(order),
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def _finish(proc, timeout):
    try:
        out, err = proc.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        proc.kill()
        out, err = proc.communicate()
        raise AssertionError(f"timed out\n{out[-6000:]}")
    text = out + "\n".join(l for l in err.splitlines() if "makecontext" not in l)
    assert proc.returncode == 0 and "[emu] all passed" in out, text[-6000:]
    return text


def run_cases(cases, order="fwd", timeout=900):
    return _finish(_start(cases, order), timeout)


GROUPS = [
    (("tiny", "edges", "config0", "multirobot", "fallback_eval", "static_many_slices"), "rev"),
    (("slice_runs", "crowded_cells", "dense_tiles", "unaligned_points"), "rand"),
    (("crop", "dense", "multirobot_large"), "rand"),
    (("many_chunks", "two_level"), "fwd"),
    (("batch", "batch_resident", "batch_mixed_radius", "batch_tune"), "rand"),
    (("traj_value_grad", "autotune"), "fwd"),
    (("plan", "unique"), "rand"),
    (("plan_query",), "fwd"),
    (("insert", "traj_opt"), "rev"),
]


@pytest.fixture(scope="module")
def running(emu_lib):
    """All groups start at once, each in its own process (one core each)."""
    procs = {g: _start(list(g[0]), g[1]) for g in GROUPS}
    yield procs
    for p in procs.values():
        if p.poll() is None:
            p.kill()
            p.communicate()


@pytest.mark.parametrize("group", GROUPS, ids=["+".join(g[0]) for g in GROUPS])
def test_kernels_on_cpu(running, group):
    _finish(running[group], timeout=1200)


@pytest.mark.skipif(os.environ.get("PCT_EMU_FULL") != "1", reason="full-size map on the CPU build takes minutes; "
                    "set PCT_EMU_FULL=1")
def test_full_size_map_on_cpu(emu_lib):
    run_cases(["config1_build"], "fwd", timeout=3000)

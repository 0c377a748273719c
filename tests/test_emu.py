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


def run_cases(cases, order="fwd", timeout=900):
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_emu.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["EMU_ORDER"] = order
    env["OMP_NUM_THREADS"] = env.get("OMP_NUM_THREADS", "4")
    r = subprocess.run([sys.executable, os.path.join(EMU, "driver.py"), *cases], env=env, capture_output=True,
                       text=True, timeout=timeout)
    out = r.stdout + "\n".join(l for l in r.stderr.splitlines() if "makecontext" not in l)
    assert r.returncode == 0 and "[emu] all passed" in r.stdout, out[-6000:]
    return out


@pytest.mark.parametrize("cases,order", [
    (["tiny", "edges", "config0", "multirobot", "fallback_eval"], "rev"),
    (["crop", "dense", "multirobot_large"], "rand"),
    (["many_chunks", "two_level"], "fwd"),
    (["batch", "batch_resident", "batch_mixed_radius"], "rand"),
    (["traj_value_grad", "autotune"], "fwd"),
    (["plan"], "rand"),
])
def test_kernels_on_cpu(emu_lib, cases, order):
    run_cases(cases, order)


@pytest.mark.skipif(os.environ.get("PCT_EMU_FULL") != "1", reason="full-size map on the CPU build takes minutes; "
                    "set PCT_EMU_FULL=1")
def test_full_size_map_on_cpu(emu_lib):
    run_cases(["config1_build"], "fwd", timeout=3000)

"""The host C++ under AddressSanitizer with UndefinedBehaviorSanitizer and under ThreadSanitizer, and the batched solver's body
logic (isb_body.hpp, run by host threads as emulated workgroups of 2 and 4 waves, with its debug
index checks) under ThreadSanitizer and under AddressSanitizer with UndefinedBehaviorSanitizer. CPU only: the sanitized libraries are built with g++ from the same sources
(the host-only isb_host.cpp; the emulator of tests/emu) and driven by tests/san_driver.py in a child
process with the sanitizer runtime preloaded, so that a report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_05791_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
BUILD = os.path.join(EMU, "_build")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is needed for the sanitizer builds")


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} not available")
    return p


def _build(out, srcs, flags, deps):
    os.makedirs(BUILD, exist_ok=True)
    if os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(d) for d in deps):
        return out
    tmp = f"{out}.{os.getpid()}.tmp"  # parallel test workers build apart, then one rename wins
    cmd = ["g++", "-O1", "-g", "-fPIC", "-shared", "-fno-omit-frame-pointer", *flags, *srcs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    os.replace(tmp, out)
    return out


def _drive(mode, lib, runtime, env_extra, timeout):
    env = dict(os.environ, LD_PRELOAD=runtime, OMP_NUM_THREADS="1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "tests.san_driver", mode, lib], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=timeout)
    report = r.stdout[-2000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in r.stderr, report
    return r.stdout


def test_host_abi_under_asan_and_ubsan():
    src = os.path.join(CSRC, "isb_host.cpp")
    lib = _build(os.path.join(BUILD, "libisb_host_asan.so"), [src],
                 ["-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                 [src, os.path.join(CSRC, "isb_host.hpp"), os.path.join(ROOT, "include", "isb.h")])
    out = _drive("host", lib, _runtime("libasan.so"), {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                                                       "UBSAN_OPTIONS": "print_stacktrace=1"}, 300)
    assert "host ABI checks passed" in out


def test_host_abi_under_tsan():
    """The host library under ThreadSanitizer: isb_wave_order balances its patches on threads."""
    src = os.path.join(CSRC, "isb_host.cpp")
    lib = _build(os.path.join(BUILD, "libisb_host_tsan.so"), [src], ["-std=c++17", "-pthread", "-fsanitize=thread"],
                 [src, os.path.join(CSRC, "isb_host.hpp"), os.path.join(ROOT, "include", "isb.h")])
    out = _drive("host", lib, _runtime("libtsan.so"), {"TSAN_OPTIONS": "halt_on_error=1:exitcode=66"}, 300)
    assert "host ABI checks passed" in out


@pytest.mark.slow
def test_emulated_batched_solver_under_tsan():
    from tests.emu import emu
    src = os.path.join(EMU, "batched_emu.cpp")
    lib = _build(os.path.join(BUILD, "libisb_emu_tsan.so"), [src],
                 ["-std=c++20", "-pthread", "-fsanitize=thread", "-DISB_DEBUG", "-I", os.path.join(EMU, "include"),
                  "-I", CSRC], emu.SRCS)
    out = _drive("emu", lib, _runtime("libtsan.so"), {"TSAN_OPTIONS": "halt_on_error=1:exitcode=66"}, 900)
    assert "emulated batched solver checks passed" in out


@pytest.mark.slow
def test_emulated_batched_solver_under_asan_and_ubsan():
    """The same emulated runs with AddressSanitizer and UndefinedBehaviorSanitizer: every access of
    the body logic to the element, vertex and LDS arrays stays inside its allocation."""
    from tests.emu import emu
    src = os.path.join(EMU, "batched_emu.cpp")
    lib = _build(os.path.join(BUILD, "libisb_emu_asan.so"), [src],
                 ["-std=c++20", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-DISB_DEBUG", "-I", os.path.join(EMU, "include"), "-I", CSRC], emu.SRCS)
    out = _drive("emu", lib, _runtime("libasan.so"), {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                                                      "UBSAN_OPTIONS": "print_stacktrace=1"}, 900)
    assert "emulated batched solver checks passed" in out

"""The library's host logic under AddressSanitizer and ThreadSanitizer, on
the CPU.

The runtime is compiled host-only (no kernels) with AddressSanitizer and
linked against a stand-in for the HIP runtime (``asan_hip_stub.cpp``) whose
device memory is host memory, so every upload, copy and fill the library
issues is a checked access to the allocation it targets.  The replay
(``asan_replay_driver.cpp``) runs the batch autotuner's whole candidate
sequence over the square m = 2..14 sweep, graph-mode strips with one to
three chunk groups, resident strips in both arithmetic forms and the strip
that allocates nothing.  A second build turns the batch's chunk groups back
on (they are switched off in the product), so their stage-table layout and
fork/join are replayed too.  Under ThreadSanitizer, ``tsan_replay_driver.cpp``
builds the coefficient form's host maps on a second thread while the main
thread runs coefficient-form strips (the concurrent use that preceded a
crash in Python's garbage collector on the GPU machine): no data race may be
reported.  ``tsan_capture_driver.cpp`` has three threads capture graph-mode,
grouped and coefficient-form strips at once; the stand-in aborts when a
capture begins on a stream that is already capturing.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_1005_3609_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
GROUPS_OFF = "  bp.groups = 1;\n"
GROUPS_ON = "  bp.groups = std::max(1, std::min(t.streams, 4));\n"


def _san_runtime(kind="asan"):
    try:
        p = subprocess.run([CLANG, f"-print-file-name=libclang_rt.{kind}-x86_64.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isfile(p) else None


def _run(cmd, cwd, env=None, timeout=600):
    r = subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...: rc {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


def _build(top, san, groups_on, driver):
    """Builds the host-only library with sanitizer `san` and `driver`; returns
    (build dir, driver path)."""
    # the sources include the public header as ../../include/chromstrip.h
    tmp = os.path.join(top, "pkg", "csrc")
    os.makedirs(tmp)
    os.symlink(os.path.join(ROOT, "include"), os.path.join(top, "include"))
    src = open(os.path.join(CSRC, "runtime.hip")).read()
    if groups_on:
        assert src.count(GROUPS_OFF) == 1, "the batch plan's chunk-group line moved; update this test"
        src = src.replace(GROUPS_OFF, GROUPS_ON)
    for f in os.listdir(CSRC):
        if f.endswith((".hpp", ".cpp")):
            shutil.copy(os.path.join(CSRC, f), tmp)
    with open(os.path.join(tmp, "runtime.hip"), "w") as fh:
        fh.write(src)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", tmp]
    host = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC"]
    flag = f"-fsanitize={san}"
    _run([HIPCC, "-x", "hip", "--cuda-host-only", *host, *inc, "-Xarch_host", flag, "-c",
          "runtime.hip", "-o", "runtime.o"], tmp)
    fat = [ln.split()[-1] for ln in _run(["nm", "-u", "runtime.o"], tmp).stdout.splitlines()
           if "__hip_fatbin" in ln]
    assert len(fat) == 1, fat
    for f in ("states", "maps"):
        _run([CLANG, *host, flag, *inc, "-c", f"{f}.cpp", "-o", f"{f}.o"], tmp)
    _run([CLANG, *host, flag, f"-DHIP_FATBIN_SYMBOL={fat[0]}", "-I", "/opt/rocm/include", "-c",
          os.path.join(HERE, "asan_hip_stub.cpp"), "-o", "stub.o"], tmp)
    _run([CLANG, "-shared", flag, "-shared-libsan", "-o", "libreplay.so", "runtime.o", "states.o",
          "maps.o", "stub.o", "-lpthread"], tmp)
    _run([CLANG, *host, flag, "-shared-libsan", "-Wno-unused-result", "-D__HIP_PLATFORM_AMD__",
          *inc, "-I", "/opt/rocm/include", os.path.join(HERE, driver), "-o", "replay", "-L", tmp,
          "-lreplay", f"-Wl,-rpath,{tmp}", "-lpthread"], tmp)
    return tmp, os.path.join(tmp, "replay")


def _env(kind, options):
    env = dict(os.environ, LD_LIBRARY_PATH=os.path.dirname(_san_runtime(kind)) + ":" +
               os.environ.get("LD_LIBRARY_PATH", ""))
    env[f"{kind.upper()}_OPTIONS"] = options
    env.pop("LD_PRELOAD", None)
    return env


def _build_and_replay(top, groups_on):
    tmp, exe = _build(top, "address", groups_on, "asan_replay_driver.cpp")
    r = _run([exe, "1"], tmp, env=_env("asan", "detect_leaks=0:abort_on_error=0"), timeout=900)
    lines = r.stdout.splitlines()
    assert lines[-1] == "done"
    assert sum(ln.startswith("batch ") for ln in lines) == 48
    assert sum(ln.startswith("graph strip") for ln in lines) == 18
    assert sum(ln.startswith("resident") for ln in lines) == 8
    assert sum(ln.startswith("split strip") for ln in lines) == 8
    assert "ERROR: AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or _san_runtime("asan") is None,
                    reason="needs hipcc and clang's AddressSanitizer runtime")
@pytest.mark.parametrize("groups_on", [False, True], ids=["as_built", "batch_chunk_groups_on"])
def test_host_logic_is_clean_under_asan(tmp_path, groups_on):
    _build_and_replay(str(tmp_path), groups_on)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or _san_runtime("tsan") is None,
                    reason="needs hipcc and clang's ThreadSanitizer runtime")
def test_concurrent_host_map_builds_are_race_free_under_tsan(tmp_path):
    tmp, exe = _build(str(tmp_path), "thread", False, "tsan_replay_driver.cpp")
    for lat, m_hi in ((0, 13), (1, 11)):
        r = _run([exe, str(lat), str(m_hi)], tmp, env=_env("tsan", "halt_on_error=1"), timeout=900)
        assert r.stdout.splitlines()[-1] == "done"
        assert sum(ln.startswith("series m") for ln in r.stdout.splitlines()) == m_hi
        assert "WARNING: ThreadSanitizer" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or _san_runtime("tsan") is None,
                    reason="needs hipcc and clang's ThreadSanitizer runtime")
def test_concurrent_graph_captures_are_serialised(tmp_path):
    # three host threads capture graph-mode, grouped and coefficient-form
    # strips at once; the stand-in aborts if two captures overlap on one stream
    tmp, exe = _build(str(tmp_path), "thread", False, "tsan_capture_driver.cpp")
    r = subprocess.run([exe, "6"], cwd=tmp, env=_env("tsan", "halt_on_error=1"), capture_output=True, text=True,
                       timeout=900)
    assert "already capturing" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, f"rc {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    assert r.stdout.splitlines()[-1] == "done"
    assert "WARNING: ThreadSanitizer" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or _san_runtime("asan") is None,
                    reason="needs hipcc and clang's AddressSanitizer runtime")
def test_repeated_batch_is_captured_once(tmp_path):
    # the cached batch graph is keyed by what its launches capture; bytes the
    # launches never read (padding, unused union members) must not make an
    # identical batch miss the cache and be captured again
    tmp, exe = _build(str(tmp_path), "address", False, "asan_batch_cache_driver.cpp")
    r = _run([exe], tmp, env=_env("asan", "detect_leaks=0:abort_on_error=0"), timeout=600)
    assert r.stdout.splitlines()[-1] == "captures 1", r.stdout[-500:]

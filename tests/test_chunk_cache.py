"""Host logic of the device chunk cache (csrc/chunk_cache.h): the ownership
ledger and the completion-token rule, under 16 host threads and a simulated
device, built three ways: plain, with ThreadSanitizer on the host code, and
with the token rule removed (which the check must catch)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chunk_cache_check.cc")


def _build_run(tmp_path, name, extra):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-pthread", *extra, SRC, "-o", exe],
                   check=True, capture_output=True, text=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    return r.returncode, r.stdout + r.stderr


def test_ledger_and_tokens(tmp_path):
    rc, out = _build_run(tmp_path, "ok", ["-Wall", "-Wextra", "-Werror"])
    assert rc == 0 and "OK" in out, out


def test_ledger_and_tokens_thread_sanitizer(tmp_path):
    rc, out = _build_run(tmp_path, "tsan", ["-fsanitize=thread"])
    assert rc == 0 and "ThreadSanitizer" not in out, out


def test_ignoring_tokens_is_caught(tmp_path):
    rc, out = _build_run(tmp_path, "mut", ["-DIGNORE_TOKENS"])
    assert rc == 0 and "violation detected" in out, out

"""The committed rocprofv3 summaries under profiles/ describe the current kernels.

Each summary names the kernel sources it was taken with and a SHA-256 prefix of their
bytes (in the listed order); a kernel change without new profiles fails here.
"""
import hashlib
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2105_04150_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def _summaries():
    return sorted(f for f in os.listdir(PROFILES) if f.endswith(".txt"))


def _field(lines, key):
    for ln in lines:
        if ln.startswith(key + ":"):
            return ln.split(":", 1)[1].strip()
    return None


def test_every_summary_carries_its_command():
    names = _summaries()
    assert names, "no profile summaries"
    for name in names:
        lines = open(os.path.join(PROFILES, name)).read().splitlines()
        assert any(ln.startswith("command") and "rocprofv3" in ln for ln in lines), name


@pytest.mark.parametrize("name", _summaries())
def test_summary_matches_kernel_sources(name):
    lines = open(os.path.join(PROFILES, name)).read().splitlines()
    files = _field(lines, "kernel_source_files")
    want = _field(lines, "kernel_source_sha256_16")
    assert files and want, f"{name}: no kernel source hash"
    h = hashlib.sha256()
    for f in files.split():
        h.update(open(os.path.join(CSRC, os.path.basename(f)), "rb").read())
    assert h.hexdigest()[:16] == want, f"{name} was taken with other kernel sources"

"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/gbd.h declares, and fails cleanly (no crash) without a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from gbd_testutil import ensure_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gbd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gbd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("gbd_beamlets", "gbd_plane", "gbd_eval", "gbd_ctx_create", "gbd_plan_setup", "gbd_plan_eval"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ensure_library())
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_names_match_abi():
    import paper_2404_12454_amd as g
    for name in ("gbd_ctx_create", "gbd_beamlets", "gbd_plane", "gbd_eval", "gbd_plan_create",
                 "gbd_plan_setup", "gbd_plan_eval", "gbd_plan_shape"):
        assert callable(getattr(g, name))


def test_context_creation_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    code = (
        "import ctypes, sys\n"
        f"lib = ctypes.CDLL({ensure_library()!r})\n"
        "lib.gbd_last_error.restype = ctypes.c_char_p\n"
        "h = ctypes.c_void_p()\n"
        "rc = lib.gbd_ctx_create(ctypes.byref(h), 0, None)\n"
        "print(rc, lib.gbd_last_error().decode())\n"
        "sys.exit(0 if rc < 0 and h.value is None else 1)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr

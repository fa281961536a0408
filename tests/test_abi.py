"""The C-ABI library loads and exports every entry point its header declares
(CPU: no compute call is made without a GPU)."""

import ctypes
import os
import subprocess

import pytest

import paper_2412_07127_amd as pkg


def test_library_exports_header_symbols():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libicpcg.so is not built (run __graft_entry__.build())")
    syms = pkg.declared_symbols()
    assert len(syms) >= 20
    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l and l.split()[-1].startswith("icpcg_")}
    assert exported == set(syms), exported ^ set(syms)


def test_host_only_entry_points():
    lib = pkg.load()
    assert b"gfx950" in lib.icpcg_version()
    for st in range(9):
        assert lib.icpcg_status_string(st)
    assert lib.icpcg_status_string(4) == b"maximum iterations reached"


def test_no_gpu_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    # no silent CPU path: creating a context without a device raises
    with pytest.raises(RuntimeError):
        pkg.Context()


def test_library_built_for_gfx950_only():
    """The embedded device code objects target gfx950 and nothing else."""
    blob = open(pkg.LIB_PATH, "rb").read()
    import re
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-[-a-z0-9:+]*gfx[0-9a-f]+", blob))
    assert targets, "no device code found"
    assert all(t.endswith(b"gfx950") for t in targets), targets

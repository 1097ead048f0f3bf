"""The C-ABI boundary without a GPU: the library builds and loads, exports
every entry point include/mbdp.h declares, rejects bad arguments before any
device work, and the product path neither reaches the oracle nor falls back
to the CPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2110_02901_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbdp.h")
PKG = os.path.join(ROOT, "paper_2110_02901_amd")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2110_02901_amd import build
        build.build_library()
    return binding.lib()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^(?:mbdp_status|size_t|const char\*)\s+(\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert header_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in header_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_library_is_built_for_gfx950():
    out = subprocess.run(["strings", binding.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


NULL = None
DUMMY = ctypes.c_void_p(0x1000)  # never dereferenced: argument checks come first


def test_create_dense_argument_checks(lib):
    h = ctypes.c_void_p()
    bad = [
        (0, 4, DUMMY, DUMMY, 0.9),     # n < 1
        (2**31, 4, DUMMY, DUMMY, 0.9), # n too large for int32 states
        (8, 0, DUMMY, DUMMY, 0.9),     # m < 1
        (8, 4, NULL, DUMMY, 0.9),      # P NULL
        (8, 4, DUMMY, NULL, 0.9),      # c NULL
        (8, 4, DUMMY, DUMMY, 1.0),     # gamma not < 1
        (8, 4, DUMMY, DUMMY, 0.0),     # gamma not > 0
        (8, 4, DUMMY, DUMMY, float("nan")),
    ]
    for args in bad:
        assert lib.mdp_create_dense(*args, ctypes.byref(h)) == binding.MBDP_ERR_INVALID_ARG, args
        assert not h.value
        assert binding.last_error()
    assert lib.mdp_create_dense(8, 4, DUMMY, DUMMY, 0.9, None) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mdp_create_dense(8, 2000, DUMMY, DUMMY, 0.9, ctypes.byref(h)) == \
        binding.MBDP_ERR_UNSUPPORTED
    assert "gamma" in (lib.mdp_create_dense(8, 4, DUMMY, DUMMY, 1.5, ctypes.byref(h)) and
                       binding.last_error())


def test_create_csr_argument_checks(lib):
    h = ctypes.c_void_p()
    bad = [
        (0, 2, DUMMY, DUMMY, DUMMY, 10, DUMMY, 0.9),
        (5, 0, DUMMY, DUMMY, DUMMY, 10, DUMMY, 0.9),
        (5, 2, DUMMY, DUMMY, DUMMY, -1, DUMMY, 0.9),
        (5, 2, NULL, DUMMY, DUMMY, 10, DUMMY, 0.9),
        (5, 2, DUMMY, NULL, DUMMY, 10, DUMMY, 0.9),
        (5, 2, DUMMY, DUMMY, NULL, 10, DUMMY, 0.9),
        (5, 2, DUMMY, DUMMY, DUMMY, 10, NULL, 0.9),
        (5, 2, DUMMY, DUMMY, DUMMY, 10, DUMMY, 1.0),
    ]
    for args in bad:
        assert lib.mdp_create_csr(*args, NULL, ctypes.byref(h)) == binding.MBDP_ERR_INVALID_ARG, args


def test_calls_on_a_null_handle(lib):
    st = binding.Stats()
    assert lib.mdp_workspace_bytes(NULL, 1) == 0
    name = ctypes.c_char_p()
    assert lib.mdp_engine(NULL, 1, ctypes.byref(name)) == binding.MBDP_ERR_INVALID_ARG
    assert name.value is None
    assert lib.mdp_destroy(NULL) == binding.MBDP_OK
    assert lib.mdp_set_tuning(NULL, None) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mdp_validate(NULL, 1e-6, DUMMY, 1 << 20, NULL, None) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mb_sweep(NULL, DUMMY, NULL, 1, 0, 0, NULL, NULL, NULL, DUMMY, 1 << 20, NULL) == \
        binding.MBDP_ERR_INVALID_ARG
    assert lib.vi_solve(NULL, DUMMY, NULL, NULL, 1, 0, 0, 1e-8, 0.0, NULL, 10, DUMMY, 1 << 20,
                        NULL, ctypes.byref(st)) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mpi_solve(NULL, DUMMY, NULL, DUMMY, 1, 5, 1, 0, 0, 1e-8, 0.0, NULL, 10, DUMMY,
                         1 << 20, NULL, ctypes.byref(st)) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mbdp_sync_status(NULL, 0, NULL) == binding.MBDP_ERR_WORKSPACE


def test_permutation_argument_checks(lib):
    assert lib.mbdp_permutation(0, 1, 0, DUMMY, NULL) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mbdp_permutation(10, 1, 0, NULL, NULL) == binding.MBDP_ERR_INVALID_ARG
    assert lib.mbdp_permutation(2**31, 1, 0, DUMMY, NULL) == binding.MBDP_ERR_INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(binding, "LIB_PATH", os.path.join(ROOT, "no-such-libmbdp.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.MbdpLibraryMissing):
        binding.lib()


def test_product_path_does_not_use_the_oracle():
    pattern = re.compile(r"^\s*(import|from)\s+oracle\b|oracle\.", re.M)
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pattern.search(text), os.path.join(dirpath, f)

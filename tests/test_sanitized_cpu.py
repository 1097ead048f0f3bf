"""The host runtime of libmbdp under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU needed).

A copy of the library whose host code carries both sanitizers is built
(``paper_2110_02901_amd.build_sanitized``); a child process with clang's
ASan runtime preloaded drives every entry point through its argument checks
and, where the checks pass, into the first HIP call (which fails without a
GPU and must map to MBDP_ERR_HIP with a message).  The child must end
normally with no sanitizer report."""
import os
import subprocess
import sys

import pytest

DRIVER = r"""
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
DUMMY = P(0x1000)
NULL = None
L.mbdp_last_error.restype = ctypes.c_char_p
L.mdp_workspace_bytes.restype = ctypes.c_size_t
L.mdp_batch_workspace_bytes.restype = ctypes.c_size_t
L.mdp_multi_workspace_bytes.restype = ctypes.c_size_t
for f in ("mdp_create_dense", "mdp_create_dense_q"):
    getattr(L, f).argtypes = None
L.mdp_create_dense.argtypes = [I64, I32, P, P, D, ctypes.POINTER(P)]
L.mdp_create_csr.argtypes = [I64, I32, P, P, P, I64, P, D, P, ctypes.POINTER(P)]
L.mdp_create_dense_q.argtypes = [I64, I32, P, I32, P, P, D, ctypes.POINTER(P)]
L.mdp_create_csr_q.argtypes = [I64, I32, P, P, P, I32, P, I64, P, D, P, ctypes.POINTER(P)]
L.mdp_quantize_rows.argtypes = [P, I64, I64, I32, P, P, P]
L.mbdp_permutation.argtypes = [I64, ctypes.c_uint64, ctypes.c_uint64, P, P]
L.vi_solve.argtypes = [P, P, P, P, I64, ctypes.c_uint64, ctypes.c_uint64, D, D, P, I64, P,
                       ctypes.c_size_t, P, P]
L.vi_solve_noalloc.argtypes = [P, P, P, P, I64, ctypes.c_uint64, ctypes.c_uint64, D, D, P, I64,
                               P, P]
L.mpi_solve.argtypes = [P, P, P, P, I32, I32, I64, ctypes.c_uint64, ctypes.c_uint64, D, D, P,
                        I64, P, ctypes.c_size_t, P, P]
L.mdp_refine.argtypes = [P, P, P, I32, I64, ctypes.c_uint64, ctypes.c_uint64, D, P, I64, P,
                         ctypes.c_size_t, P, P]
L.mb_sweep.argtypes = [P, P, P, I64, ctypes.c_uint64, ctypes.c_uint64, P, P, P, P,
                       ctypes.c_size_t, P]
L.mdp_multi_solve.argtypes = [P, I32, P, P, P, I64, ctypes.c_uint64, ctypes.c_uint64, D, I64, P,
                              ctypes.c_size_t, P, P]
L.mdp_batch_upload.argtypes = [P, I32, P, ctypes.c_size_t, P]
L.mdp_batch_launch.argtypes = [I32, D, I64, P, ctypes.c_size_t, P]
L.mdp_batch_read_stats.argtypes = [P, I32, P, P]
L.mdp_validate.argtypes = [P, D, P, ctypes.c_size_t, P, P]
L.mdp_policy_transpose.argtypes = [P, P, P, P, P, P, ctypes.c_size_t, P]
L.mdp_value_gradients.argtypes = [P, P, P, P, P, P, P, ctypes.c_size_t, P]
L.mdp_engine.argtypes = [P, I64, ctypes.POINTER(ctypes.c_char_p)]
L.mdp_workspace_bytes.argtypes = [P, I64]
L.mdp_multi_workspace_bytes.argtypes = [P, I32, I64]
L.mbdp_sync_status.argtypes = [P, ctypes.c_size_t, P]
OK, INV, UNS, WS, HIP = 0, 1, 2, 3, 4
checks = 0
def expect(got, want, what):
    global checks
    if got not in want:
        raise SystemExit("%s: status %d, expected %s (%s)" % (what, got, want, L.mbdp_last_error()))
    if got != OK and not L.mbdp_last_error():
        raise SystemExit("%s: no message" % what)
    checks += 1
h = P()
for args in [(0, 4, DUMMY, DUMMY, 0.9), (2**31, 4, DUMMY, DUMMY, 0.9), (8, 0, DUMMY, DUMMY, 0.9),
             (8, 4, NULL, DUMMY, 0.9), (8, 4, DUMMY, NULL, 0.9), (8, 4, DUMMY, DUMMY, 1.0),
             (8, 4, DUMMY, DUMMY, float("nan"))]:
    expect(L.mdp_create_dense(*args, ctypes.byref(h)), (INV,), "create_dense %s" % (args,))
expect(L.mdp_create_dense(8, 2000, DUMMY, DUMMY, 0.9, ctypes.byref(h)), (UNS,), "m too large")
# valid arguments reach the device query, which fails without a GPU
expect(L.mdp_create_dense(8, 4, DUMMY, DUMMY, 0.9, ctypes.byref(h)), (HIP, UNS), "no GPU")
for args in [(0, 2, DUMMY, DUMMY, DUMMY, 10, DUMMY, 0.9), (5, 2, DUMMY, DUMMY, DUMMY, -1, DUMMY, 0.9),
             (5, 2, NULL, DUMMY, DUMMY, 10, DUMMY, 0.9), (5, 2, DUMMY, DUMMY, DUMMY, 10, DUMMY, 2.0)]:
    expect(L.mdp_create_csr(*args, NULL, ctypes.byref(h)), (INV,), "create_csr %s" % (args,))
expect(L.mdp_create_dense_q(16, 2, DUMMY, 7, DUMMY, DUMMY, 0.9, ctypes.byref(h)), (INV, UNS),
       "dense_q bad dtype")
expect(L.mdp_create_dense_q(12, 2, DUMMY, 1, DUMMY, DUMMY, 0.9, ctypes.byref(h)), (INV, UNS),
       "dense_q n % 8")
expect(L.mdp_create_csr_q(5, 2, DUMMY, DUMMY, DUMMY, 1, DUMMY, -3, DUMMY, 0.9, NULL,
                          ctypes.byref(h)), (INV,), "csr_q nnz")
expect(L.mdp_quantize_rows(NULL, 4, 4, 1, DUMMY, DUMMY, NULL), (INV,), "quantize NULL")
expect(L.mdp_quantize_rows(DUMMY, 4, 4, 9, DUMMY, DUMMY, NULL), (INV, UNS), "quantize dtype")
expect(L.mbdp_permutation(0, 1, 0, DUMMY, NULL), (INV,), "perm n")
expect(L.mbdp_permutation(10, 1, 0, NULL, NULL), (INV,), "perm out")
st = ctypes.create_string_buffer(256)
expect(L.vi_solve(NULL, DUMMY, NULL, NULL, 1, 0, 0, 1e-8, 0.0, NULL, 10, DUMMY, 1 << 20, NULL, st),
       (INV,), "vi_solve NULL")
expect(L.vi_solve_noalloc(NULL, DUMMY, NULL, NULL, 1, 0, 0, 1e-8, 0.0, NULL, 10, NULL, st),
       (INV,), "vi_solve_noalloc NULL")
expect(L.mpi_solve(NULL, DUMMY, NULL, DUMMY, 1, 5, 1, 0, 0, 1e-8, 0.0, NULL, 10, DUMMY, 1 << 20,
                   NULL, st), (INV,), "mpi_solve NULL")
expect(L.mdp_refine(NULL, DUMMY, NULL, 0, 1, 0, 0, 1e-6, NULL, 10, DUMMY, 1 << 20, NULL, st),
       (INV,), "refine NULL")
expect(L.mb_sweep(NULL, DUMMY, NULL, 1, 0, 0, NULL, NULL, NULL, DUMMY, 1 << 20, NULL), (INV,),
       "mb_sweep NULL")
expect(L.mdp_multi_solve(NULL, 16, DUMMY, DUMMY, NULL, 1, 0, 0, 1e-8, 10, DUMMY, 1 << 20, NULL,
                         st), (INV,), "multi NULL")
expect(L.mdp_validate(NULL, 1e-6, DUMMY, 1 << 20, NULL, NULL), (INV,), "validate NULL")
expect(L.mdp_policy_transpose(NULL, DUMMY, DUMMY, DUMMY, DUMMY, DUMMY, 1 << 20, NULL), (INV,),
       "transpose NULL")
expect(L.mdp_value_gradients(NULL, DUMMY, DUMMY, DUMMY, NULL, NULL, DUMMY, 1 << 20, NULL), (INV,),
       "gradients NULL")
expect(L.mdp_batch_upload(NULL, 0, DUMMY, 1 << 20, NULL), (INV,), "batch_upload count")
expect(L.mdp_batch_launch(0, 1e-8, 10, DUMMY, 1 << 20, NULL), (INV,), "batch_launch count")
expect(L.mdp_batch_read_stats(NULL, 1, NULL, NULL), (INV, WS), "batch stats NULL")
expect(L.mbdp_sync_status(NULL, 0, NULL), (WS,), "sync NULL")
name = ctypes.c_char_p()
expect(L.mdp_engine(NULL, 1, ctypes.byref(name)), (INV,), "engine NULL")
assert L.mdp_workspace_bytes(NULL, 1) == 0
assert L.mdp_multi_workspace_bytes(NULL, 16, 1) == 0
assert L.mdp_batch_workspace_bytes(0) == 0 and L.mdp_batch_workspace_bytes(5) > 0
assert L.mdp_destroy(NULL) == OK
print("driver-ok %d checks" % checks)
"""


def test_host_runtime_under_sanitizers():
    from paper_2110_02901_amd import build_sanitized as bs
    lib = bs.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=bs.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("HIP_VISIBLE_DEVICES", None)
    r = subprocess.run([sys.executable, "-c", DRIVER, lib], env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "driver-ok" in r.stdout, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]

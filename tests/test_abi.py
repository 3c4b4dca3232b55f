"""The C-ABI library loads and exports every symbol include/ensei.h declares,
and the comparison library every symbol of include/ensei_bench.h (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2003_05328_amd import ensei

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ensei.h")
BENCH_HEADER = os.path.join(ROOT, "include", "ensei_bench.h")
BFV_HEADER = os.path.join(ROOT, "include", "ensei_bfv.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ensei_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for core in ("ensei_ntt2d", "ensei_intt2d", "ensei_encrypt", "ensei_homconv", "ensei_decrypt"):
        assert core in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ensei.LIB_PATH):
        from paper_2003_05328_amd import build

        build.build()
    return ensei.lib()


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in ensei.SIGNATURES, f"binding lacks {name}"
    assert set(ensei.SIGNATURES) == set(declared_functions())


def test_packed_calls_are_exported(lib):
    from paper_2003_05328_amd import ensei_bfv

    names = declared_functions(BFV_HEADER)
    assert set(names) == set(ensei_bfv.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", ensei.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in names:
        assert name in exported, name
    l = ensei_bfv._lib()
    h = ctypes.c_void_p()
    # host-side refusals need no GPU: bad n, composite or ill-sized moduli, null arguments
    assert l.ensei_bfv_ctx_create(None, 12289, 8380417, 4005889, 2048, 0) == -1
    assert l.ensei_bfv_ctx_create(ctypes.byref(h), 12289, 8380417, 4005889, 48, 0) == -1
    assert l.ensei_bfv_ctx_create(ctypes.byref(h), 12289, 8380417, 4005889, 8192, 0) == -1  # n > 4096
    assert l.ensei_bfv_ctx_create(ctypes.byref(h), 12289, 8380417, 4005889, 4096, 0) == -3  # 8192 does not divide t - 1
    assert l.ensei_bfv_ctx_create(ctypes.byref(h), 12291, 8380417, 4005889, 2048, 0) == -3
    assert l.ensei_bfv_ctx_create(ctypes.byref(h), 12289, 8380417, 8380417, 2048, 0) == -3
    assert l.ensei_bfv_ctx_destroy(None) == 0
    assert l.ensei_bfv_vectors(None, 3, 1024) == 0
    assert l.ensei_bfv_key(None, None, None, None) == -1


def test_bench_library_exports_its_header(lib):
    names = declared_functions(BENCH_HEADER)
    assert names == sorted(ensei.BENCH_SIGNATURES)
    bl = ensei.bench_lib()
    for name in names:
        assert hasattr(bl, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ensei.BENCH_LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported
    # the comparison kernel is not part of the product library
    prod = subprocess.run(["nm", "-D", "--defined-only", ensei.LIB_PATH], capture_output=True, text=True,
                          check=True).stdout
    assert "homconv_valu" not in prod


def test_exports_are_unmangled_c_symbols(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", ensei.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared_functions():
        assert name in exported, name


def test_status_strings_and_host_only_calls(lib):
    for code in list(ensei.STATUS) + [0]:
        s = lib.ensei_status_str(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.ensei_status_str(12345) == b"unknown status"
    # packed-weight size is pure host arithmetic:
    # F * ceil(Cin/64) * ceil(Cout/64) * U * 16, U = 768 (Cin >= 48) or 256 * ceil(Cin/16)
    assert lib.ensei_wpack_bytes(64, 64, 1024) == 1024 * 1 * 1 * 768 * 16
    assert lib.ensei_wpack_bytes(8, 3, 256) == 256 * 1 * 1 * 256 * 16
    assert lib.ensei_wpack_bytes(40, 130, 16) == 16 * 3 * 1 * 768 * 16
    assert lib.ensei_wpack_bytes(130, 33, 5) == 5 * 1 * 3 * 768 * 16
    assert lib.ensei_wpack_bytes(512, 256, 16) == 16 * 4 * 8 * 768 * 16
    assert lib.ensei_wpack_bytes(0, 3, 256) == 0
    # context accessors tolerate NULL
    assert lib.ensei_ctx_modulus(None) == 0 and lib.ensei_ctx_delta(None) == 0
    assert lib.ensei_ctx_destroy(None) == 0


def test_entry_points_reject_null_context(lib):
    # argument checks run on the host before any HIP call touches a device
    assert lib.ensei_ntt2d(None, None, None, 1, 16, 16, None) < 0
    assert lib.ensei_homconv(None, None, None, None, 1, 1, 1, 1, 1, None, None) < 0
    assert lib.ensei_encrypt(None, None, None, None, 1, 1, 1, 1, 0, 0, None, None) < 0
    assert lib.ensei_decrypt(None, None, None, 1, 1, 1, 1, None, None) < 0
    h = ctypes.c_void_p()
    assert lib.ensei_ctx_create(None, 65537, 0) == -1  # ENSEI_ERR_ARG
    # batched plans
    assert lib.ensei_plan_create(None, None, 1, None, ctypes.byref(h)) < 0
    assert lib.ensei_plan_run(None, None) == -1
    assert lib.ensei_plan_schedule(None, None) == -1
    assert lib.ensei_plan_destroy(None) == 0


def test_server_host_checks(lib):
    h = ctypes.c_void_p()
    assert lib.ensei_server_create(None, 1 << 20, 1, 1, ctypes.byref(h)) < 0
    assert lib.ensei_server_destroy(None) == 0
    assert lib.ensei_server_submit(None, 0, None, None) == -1
    assert lib.ensei_server_wait(None, 1, 0) == -1
    assert lib.ensei_server_stats(None, None) == -1
    # a request's device footprint: x^, ct_in, ct_out, m, each 256-byte aligned
    sh = ensei.ShapeDesc(32, 32, 64, 64, 3, 3, 1024)
    F = 32 * 32
    al = lambda v: (v + 255) // 256 * 256
    assert lib.ensei_request_bytes(ctypes.byref(sh)) == al(F * 64 * 4) + 2 * al(F * 1025 * 64 * 8) + al(F * 64 * 4)
    sh.n = 0
    assert lib.ensei_request_bytes(ctypes.byref(sh)) == 0
    assert ctypes.sizeof(ensei.RequestDesc) == 8 * 8
    assert ctypes.sizeof(ensei.RequestInfo) == 8 + 3 * 8
    assert ctypes.sizeof(ensei.ServerInfo) == 10 * 8
    assert lib.ensei_server_cancel(None, 1) == -1
    assert lib.ensei_server_set_queue_limit(None, 0) == -1
    assert lib.ensei_server_clock(None, None) == -1
    assert lib.ensei_ctx_device(None) == -1


def test_plan_structs_match_the_header():
    # ensei_layer: 7 ints, int64 batch, uint64 seed_a, 11 pointers
    assert ctypes.sizeof(ensei.LayerDesc) == 7 * 4 + 4 + 8 + 8 + 11 * 8
    assert ensei.LayerDesc.batch.offset == 32 and ensei.LayerDesc.w.offset == 48
    assert ctypes.sizeof(ensei.ScheduleDesc) == 56


def test_modulus_rejected_before_device_use(lib):
    h = ctypes.c_void_p()
    assert lib.ensei_ctx_create(ctypes.byref(h), 65535, 0) == -3  # not prime
    assert lib.ensei_ctx_create(ctypes.byref(h), 1 << 22 | 1, 0) == -3  # too large
    assert lib.ensei_ctx_create(ctypes.byref(h), 2, 0) == -3
    assert h.value is None

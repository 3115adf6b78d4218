"""The C-ABI boundary on a machine without a GPU: libphos.so loads, exports
every function include/phos.h declares, the ctypes binding names exactly
those functions, and the argument checks the header documents return their
status before any device work.  No call here reaches the HIP runtime: the
handle-first entry points are called with a NULL handle, and phos_create
with arguments it rejects before it looks for a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phos.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return {m.group(1) for m in re.finditer(r"\b(phos_[a-z0-9_]+)\s*\(", text)}


@pytest.fixture(scope="module")
def phos():
    from paper_2405_12079_amd import phos as p
    return p


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("phos_create", "phos_destroy", "phos_buffers_register", "phos_spec_register",
                 "phos_spec_release", "phos_validate", "phos_validate_batch", "phos_ckpt_begin",
                 "phos_ckpt_cow", "phos_ckpt_recopy", "phos_ckpt_end", "phos_restore_begin",
                 "phos_restore_on_demand", "phos_restore_end", "phos_copy_batch",
                 "phos_copy_batch_tuned", "phos_stream_status", "phos_manifest_write",
                 "phos_manifest_check", "phos_last_error"):
        assert core in names, core


def test_library_exports_every_declared_function(phos):
    out = subprocess.run(["nm", "-D", "--defined-only", phos.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = _declared() - exported
    assert not missing, f"declared in phos.h but not exported: {sorted(missing)}"
    lib = ctypes.CDLL(phos.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_the_header(phos):
    bound = {name for name, _ in phos.SIGNATURES} | {"phos_last_error"}
    assert bound == _declared()


def _zero(t):
    if t is ctypes.c_char_p:
        return None
    if isinstance(t, type) and issubclass(t, ctypes._Pointer):
        return None
    return t(0)


def test_null_handles_are_rejected(phos):
    """Every entry point whose first argument is a handle returns E_INVAL for
    a NULL one (and says why in phos_last_error)."""
    lib = phos.lib()
    checked = 0
    for name, args in phos.SIGNATURES:
        if args[0] is not ctypes.c_void_p:
            continue
        st = getattr(lib, name)(*[_zero(t) for t in args])
        assert st == phos.E_INVAL, f"{name}: status {st}"
        assert lib.phos_last_error(), name
        checked += 1
    assert checked >= 30


@pytest.mark.parametrize("base,nbytes,page,why", [
    (1 << 30, 1 << 30, 3000, "page_bytes"),           # not a power of two
    (1 << 30, 1 << 30, 2048, "page_bytes"),           # below 4 KiB
    (1 << 30, 1 << 30, 4 << 20, "page_bytes"),        # above 2 MiB
    ((1 << 30) + 4096, 1 << 30, 65536, "multiples"),  # base not page aligned
    (1 << 30, (1 << 30) + 4096, 65536, "multiples"),  # size not whole pages
    (0, 1 << 30, 65536, "multiples"),                 # no pool
    ((1 << 64) - (1 << 20), 1 << 30, 4096, "wraps"),  # pool runs past 2^64
])
def test_create_rejects_bad_pools(phos, base, nbytes, page, why):
    lib = phos.lib()
    out = ctypes.c_void_p(1)
    st = lib.phos_create(0, base, nbytes, page, ctypes.byref(out))
    assert st == phos.E_INVAL
    assert out.value is None
    assert why in lib.phos_last_error().decode()


def test_create_rejects_null_out(phos):
    assert phos.lib().phos_create(0, 1 << 30, 1 << 30, 65536, None) == phos.E_INVAL


def test_status_codes_and_flags_match_the_header(phos):
    """The binding's constants are the header's values (E_OVERFLOW and
    E_MISSPEC included, which asynchronous calls report later)."""
    text = open(HEADER).read()
    for name, val in (("PHOS_E_OVERFLOW", phos.E_OVERFLOW), ("PHOS_E_MISSPEC", phos.E_MISSPEC),
                      ("PHOS_E_TIMEOUT", phos.E_TIMEOUT), ("PHOS_V_SYNC", phos.V_SYNC),
                      ("PHOS_V_TRACK", phos.V_TRACK)):
        m = re.search(name + r"\s*=\s*(\d+)u?", text)
        assert m and int(m.group(1)) == val, name


def test_manifest_and_batch_calls_check_before_device_work(phos):
    lib = phos.lib()
    n = ctypes.c_uint64(0)
    assert lib.phos_manifest_write(None, 1, None, 0, ctypes.byref(n)) == phos.E_INVAL
    assert lib.phos_manifest_check(None, b"PHOSIMG1", 8) == phos.E_INVAL
    assert lib.phos_copy_batch(None, None, 0, None) == phos.E_INVAL
    assert lib.phos_copy_batch_tuned(None, None, 0, None) == phos.E_INVAL
    assert lib.phos_stream_status(None, None) == phos.E_INVAL

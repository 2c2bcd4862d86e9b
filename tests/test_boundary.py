"""Host-side checks of the C ABI boundary (no device calls): the library
loads and exports every function that include/spamm.h declares, and the
binding's structure layouts match the header's."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spamm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*([a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("spamm_tree_build", "spamm_multiply", "sp2_solve", "spamm_cull",
                 "spamm_to_dense", "spamm_matrix_destroy", "spamm_last_error"):
        assert must in names


def test_library_loads_and_exports_every_declared_symbol():
    import paper_1403_7458_amd as sp
    lib = sp.load()
    out = subprocess.run(["nm", "-D", "--defined-only", sp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    # The binding describes exactly the declared functions.
    assert set(sp.SIGNATURES) == set(declared_functions())
    assert sp.version().startswith("spamm-mi355x")


def test_struct_sizes_match_the_header():
    from paper_1403_7458_amd import _lib
    # Sizes implied by the field lists of include/spamm.h (x86-64 System V).
    assert ctypes.sizeof(_lib.SpammInfo) == 48
    assert ctypes.sizeof(_lib.MultStats) == 48
    assert ctypes.sizeof(_lib.Sp2Options) == 40
    assert ctypes.sizeof(_lib.Sp2Stats) == 16 + 24 + 8 + 256 + 4 * 8 * 256
    assert ctypes.sizeof(_lib.Profile) == 6 * 8 * 2 + 8
    assert ctypes.sizeof(_lib.ServerOptions) == 16
    assert ctypes.sizeof(_lib.ServerInfo) == 12 * 8


def test_server_options_defaults_and_host_side_argument_checks():
    from paper_1403_7458_amd import _lib
    lib = _lib.load()
    o = _lib.ServerOptions()
    lib.spamm_server_options_default(ctypes.byref(o))
    assert (o.max_active, o.batch_gemm, o.device, o.fill_products) == (64, 1, -1, 1 << 18)
    # Rejected before any device call: a zero budget, max_active out of range.
    h = ctypes.c_void_p(1)
    assert lib.spamm_server_create(0, ctypes.byref(o), ctypes.byref(h)) == -1
    assert h.value is None
    assert b"budget" in lib.spamm_last_error()
    o.max_active = 0
    assert lib.spamm_server_create(1 << 30, ctypes.byref(o), ctypes.byref(h)) == -1
    lib.spamm_server_destroy(None)


def test_sp2_footprint_bound():
    """Host-only arithmetic: covers the tiles of X_n and X_{n+1} (up to
    3 (ceil(n/32))^2 of them) plus dense copies of F and P, grows with n and
    with the tile size, and is 0 for invalid arguments."""
    import paper_1403_7458_amd as sp
    tile = {"fp64": 8192, "fp32": 4096, "bf16": 4096, "fp16": 4096, "bf16x3": 8192,
            "fp16x3": 8192}
    for prec, tb in tile.items():
        last = 0
        for n in (1, 31, 32, 33, 180, 750, 3750, 10000):
            rb = -(-n // 32)
            b = sp.sp2_footprint_bytes(n, prec)
            assert b >= 3 * rb * rb * tb + 2 * n * n * 8
            assert b >= last
            last = b
    # FP64 blocks are 8 KiB, BF16 ones 4 KiB; FP32 iterates hold 4 KiB blocks
    # and a column-quad copy of each.
    assert sp.sp2_footprint_bytes(3750, "fp64") > sp.sp2_footprint_bytes(3750, "bf16")
    assert sp.sp2_footprint_bytes(3750, "fp32") > sp.sp2_footprint_bytes(3750, "fp64")
    assert sp.sp2_footprint_bytes(0, "fp32") == 0
    assert sp.sp2_footprint_bytes(100, 9) == 0


def test_profile_phase_mask_checks():
    """Host-only: a phase mask must select at least one of the six phases."""
    import paper_1403_7458_amd as sp
    from paper_1403_7458_amd import _lib
    lib = _lib.load()
    assert lib.spamm_profile_phases(0) == -1
    assert lib.spamm_profile_phases(1 << 6) == -1
    assert b"mask" in lib.spamm_last_error()
    assert lib.spamm_profile_phases(1 << 3) == 0
    with pytest.raises(ValueError):
        sp.profile_phases("gemm", "nope")
    sp.profile_phases("gemm", "cull")
    sp.profile_phases()                      # back to every phase


def test_sp2_options_defaults_come_from_the_library():
    from paper_1403_7458_amd import _lib
    o = _lib.Sp2Options()
    _lib.load().sp2_options_default(ctypes.byref(o))
    assert (o.precision, o.max_iter, o.min_iter, o.stall_rule) == (1, 100, 0, 1)
    assert o.tol == 1e-8 and o.stall_floor == 0.0 and o.symmetric == 1


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_1403_7458_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "libspamm.so"))

"""The C-ABI library loads and exports every entry point include/*.h declares
(no GPU needed: nothing is launched)."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2305_04966_amd", "libtxs.so")


def declared_symbols():
    syms = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        syms |= set(re.findall(r"\b(txs_[a-z0-9_]+)\s*\(", text))
    return sorted(syms)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2305_04966_amd.build as b
        b.build()
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_covers_the_header():
    from paper_2305_04966_amd import exported_symbols
    assert set(declared_symbols()) == set(exported_symbols())


def test_version_and_error_without_gpu(lib):
    lib.txs_abi_version.restype = C.c_int32
    lib.txs_last_error.restype = C.c_char_p
    assert lib.txs_abi_version() == 2
    # argument validation happens on the host before any launch
    lib.txs_resample.restype = C.c_int32
    st = lib.txs_resample(C.c_int32(4), C.c_int32(0), None, None, C.c_int32(0), C.c_int32(8),
                          None, None, None)
    assert st == -1
    assert b"n_bins" in lib.txs_last_error()
    lib.txs_scan_workspace_size.restype = C.c_size_t
    assert lib.txs_scan_workspace_size(C.c_int32(1 << 20)) >= 8 * 256


def test_brick_occupancy_sizes(lib):
    """Two arrays of ceil((res/8)^3 / 32) words and a count word per level; no
    bricks below res 8;
    the coarsening refuses such grids on the host."""
    lib.txs_grid_coarse_words.restype = C.c_int64
    lib.txs_grid_coarse_words.argtypes = [C.c_int32]
    assert lib.txs_grid_coarse_words(4) == 0
    assert lib.txs_grid_coarse_words(8) == 2 + 1
    assert lib.txs_grid_coarse_words(64) == 2 * 16 + 1
    assert lib.txs_grid_coarse_words(128) == 2 * 128 + 1
    assert lib.txs_grid_coarse_words(1024) == 2 * 128 ** 3 // 32 + 1
    assert lib.txs_grid_coarse_words(100) == 0
    from paper_2305_04966_amd._lib import Grid
    g = Grid()
    g.bits, g.res, g.n_levels, g.half_extent0 = 1024, 4, 1, 1.5
    lib.txs_grid_coarsen.restype = C.c_int32
    assert lib.txs_grid_coarsen(C.byref(g), C.c_void_p(4096), None) == -1


def test_counts_past_int32_return_eoverflow(lib):
    """A packed tensor of 2^31 or more samples is refused with TXS_EOVERFLOW on
    the host, before any launch."""
    lib.txs_render_fwd.restype = C.c_int32
    lib.txs_last_error.restype = C.c_char_p
    big = C.c_int64(1 << 31)
    st = lib.txs_render_fwd(None, C.c_int32(0), C.c_int32(4), big, None, None, None, None, None,
                            None, None, None, None, None, None)
    assert st == -4 and b"int32" in lib.txs_last_error()
    lib.txs_transmittance_prefix.restype = C.c_int32
    st = lib.txs_transmittance_prefix(None, C.c_int32(4), big, None, None, None, C.c_float(1e-4),
                                      None, None)
    assert st == -1  # a null table is refused first
    lib.txs_weights_bwd.restype = C.c_int32
    st = lib.txs_weights_bwd(None, C.c_int32(0), C.c_int32(4), big, None, None, None, None, None,
                             None, None)
    assert st == -4
    lib.txs_hist_loss.restype = C.c_int32
    st = lib.txs_hist_loss(None, C.c_int32(4), big, None, None, None, C.c_int32(8), None, None,
                           C.c_float(1e-7), None, None, None)
    assert st == -4


def test_plain_c_consumer(lib, tmp_path):
    """The header is valid C99 under -Wall -Wextra -Werror -pedantic, the
    library links from C, and host-side validation answers without a GPU."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = os.path.join(ROOT, "tests", "cpp", "abi_consumer.c")
    exe = str(tmp_path / "abi_consumer")
    libdir = os.path.dirname(LIB)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                           "-I", os.path.join(ROOT, "include"), src, "-L", libdir, "-ltxs",
                           f"-Wl,-rpath,{libdir}", "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert out.stdout.strip() == "ok"

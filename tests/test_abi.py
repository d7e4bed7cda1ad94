"""The C ABI without a GPU: the library loads, exports what include/sat.h declares, and rejects
every invalid argument with its status code before making any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2410_16291_amd import _lib
from paper_2410_16291_amd._lib import (SAT_ERR_ARG, SAT_ERR_OVERFLOW, SAT_ERR_WINDOW, SAT_ERR_WORKSPACE, SAT_F64,
                                       SAT_OK, SAT_U8, SAT_U16, SAT_U32, SAT_U64, BatchItem)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sat.h")

# Fake device addresses: validation looks only at their values (NULL-ness, alignment, overlap).
IMG, SAT, SQ, OUT, OUT2, OUT3, WS = (0x10000000000 * k for k in range(1, 8))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(l for l in text.splitlines() if not l.strip().startswith("#"))
    return sorted(set(re.findall(r"\b([A-Za-z_]\w*)\s*\([^;{}]*\)\s*;", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "sat_build" in names and "window_sum" in names and "window_mean_std" in names
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_window_out_shape(lib):
    oh, ow = ctypes.c_int64(), ctypes.c_int64()
    for (H, W, h, w, s, exp) in [(512, 512, 32, 32, 1, (481, 481)), (8192, 8192, 64, 64, 1, (8129, 8129)),
                                 (70000, 85000, 100, 100, 1, (69901, 84901)),
                                 (70000, 85000, 250, 250, 1, (69751, 84751)),
                                 (70000, 85000, 500, 500, 1, (69501, 84501)), (10, 7, 3, 2, 4, (2, 2)),
                                 (1, 1, 1, 1, 1, (1, 1))]:
        assert lib.window_out_shape(H, W, h, w, s, ctypes.byref(oh), ctypes.byref(ow)) == SAT_OK
        assert (oh.value, ow.value) == exp
    assert lib.window_out_shape(10, 10, 11, 1, 1, ctypes.byref(oh), ctypes.byref(ow)) == SAT_ERR_WINDOW
    assert lib.window_out_shape(10, 10, 1, 1, 0, ctypes.byref(oh), ctypes.byref(ow)) == SAT_ERR_ARG
    assert lib.window_out_shape(10, 10, 1, 1, 1, None, ctypes.byref(ow)) == SAT_ERR_ARG
    assert b"window" in lib.sat_last_error()


def test_workspace_bytes(lib):
    a = lib.sat_build_workspace_bytes(512, 512, SAT_U8, 0)
    b = lib.sat_build_workspace_bytes(512, 512, SAT_U8, 1)
    assert 256 < a < b
    assert lib.sat_build_workspace_bytes(0, 5, SAT_U8, 0) == 0
    assert lib.sat_build_workspace_bytes(5, 5, SAT_U32, 0) == 0
    full = lib.sat_build_workspace_bytes(70000, 85000, SAT_U8, 0)
    assert full < 70000 * 85000          # lookback state stays below one byte per pixel


def build(lib, image=IMG, ptype=SAT_U8, H=64, W=80, ipitch=80, sat=SAT, sat_sq=None, spitch=80, ws=WS, wsb=None):
    if wsb is None:
        wsb = lib.sat_build_workspace_bytes(H, W, ptype if ptype in (SAT_U8, SAT_U16) else SAT_U8, int(bool(sat_sq)))
    return lib.sat_build(image, ptype, H, W, ipitch, sat, sat_sq, spitch, ws, wsb, None)


def test_sat_build_validation(lib):
    assert build(lib, image=None) == SAT_ERR_ARG
    assert build(lib, sat=None) == SAT_ERR_ARG
    assert build(lib, ptype=SAT_U32) == SAT_ERR_ARG
    assert build(lib, H=0) == SAT_ERR_ARG
    assert build(lib, W=0, ipitch=0, spitch=0) == SAT_ERR_ARG
    assert build(lib, ipitch=79) == SAT_ERR_ARG
    assert build(lib, spitch=79) == SAT_ERR_ARG
    assert build(lib, sat_sq=SAT) == SAT_ERR_ARG                    # identical tables
    assert build(lib, sat=IMG + 16) == SAT_ERR_ARG                  # table overlaps image
    assert build(lib, sat_sq=SAT + 8 * 100) == SAT_ERR_ARG          # squared table overlaps table
    assert build(lib, ws=None) == SAT_ERR_WORKSPACE
    assert build(lib, wsb=100) == SAT_ERR_WORKSPACE
    assert build(lib, ws=SAT + 64) == SAT_ERR_ARG                   # workspace overlaps table
    assert build(lib, ws=WS + 4) == SAT_ERR_ARG                     # misaligned workspace
    # 16-bit squares: column totals need H * 65535^2 < 2^62
    big_h = (1 << 62) // (65535 * 65535) + 1
    assert build(lib, ptype=SAT_U16, H=big_h, W=1, ipitch=1, spitch=1, sat_sq=SQ, wsb=1 << 40) in (
        SAT_ERR_OVERFLOW, SAT_ERR_ARG)


def test_sat_build_noalloc_validation(lib):
    """The entry point without a workspace argument: argument errors as sat_build, and builds whose
    workspace would exceed the library's fixed 128 MiB scratch are refused, all before any HIP
    call (so these run without a GPU)."""
    def nb(image=IMG, ptype=SAT_U8, H=64, W=80, ipitch=80, sat=SAT, sat_sq=None, spitch=80):
        return lib.sat_build_noalloc(image, ptype, H, W, ipitch, sat, sat_sq, spitch, None)
    assert nb(image=None) == SAT_ERR_ARG
    assert nb(sat=None) == SAT_ERR_ARG
    assert nb(ptype=SAT_U64) == SAT_ERR_ARG
    assert nb(H=0) == SAT_ERR_ARG
    assert nb(ipitch=79) == SAT_ERR_ARG
    assert nb(sat_sq=SAT) == SAT_ERR_ARG
    assert nb(sat=IMG + 16) == SAT_ERR_ARG
    limit = 128 << 20
    # the largest square 8-bit image whose workspace fits, and the next size up that does not
    for ptype, sq in ((SAT_U8, 0), (SAT_U16, 1)):
        fits = [n for n in range(8000, 17000, 100) if lib.sat_build_workspace_bytes(n, n, ptype, sq) <= limit]
        assert fits, ptype
        big = max(fits) + 100
        assert lib.sat_build_workspace_bytes(big, big, ptype, sq) > limit
        assert nb(ptype=ptype, H=big, W=big, ipitch=big, spitch=big, sat_sq=SQ if sq else None) == SAT_ERR_WORKSPACE
        assert b"scratch" in lib.sat_last_error()
    assert lib.sat_build_workspace_bytes(8192, 8192, SAT_U16, 1) <= limit     # 8192^2 16-bit with squares fits


def test_window_sum_validation(lib):
    def call(sat=SAT, ptype=SAT_U8, H=100, W=120, sp=120, h=10, w=10, s=1, out=OUT, ot=SAT_U32, op=111):
        return lib.window_sum(sat, ptype, H, W, sp, h, w, s, out, ot, op, None)
    assert call(sat=None) == SAT_ERR_ARG
    assert call(out=None) == SAT_ERR_ARG
    assert call(h=101) == SAT_ERR_WINDOW
    assert call(w=121) == SAT_ERR_WINDOW
    assert call(h=0) == SAT_ERR_ARG
    assert call(s=0) == SAT_ERR_ARG
    assert call(ot=SAT_F64) == SAT_ERR_ARG
    assert call(ptype=SAT_U64) == SAT_ERR_ARG
    assert call(op=110) == SAT_ERR_ARG                               # ow = 111
    assert call(out=SAT + 8) == SAT_ERR_ARG                          # out overlaps table
    # uint32 overflow: 7000^2 * 255 > 2^32 - 1, 4104^2 * 255 <= 2^32 - 1 < 4105^2 * 255
    assert call(H=8000, W=8000, sp=8000, h=7000, w=7000, op=1001) == SAT_ERR_OVERFLOW
    assert call(H=8000, W=8000, sp=8000, h=4105, w=4105, op=3896, ot=SAT_U32) == SAT_ERR_OVERFLOW
    assert call(ptype=SAT_U16, H=400, W=400, sp=400, h=300, w=300, op=101) == SAT_ERR_OVERFLOW  # 9e4 * 65535 > 2^32
    assert b"uint32" in lib.sat_last_error()


def test_window_mean_std_validation(lib):
    def call(sat=SAT, sq=SQ, s1=OUT, mean=OUT2, std=OUT3, h=4, w=4, op=97):
        return lib.window_mean_std(sat, sq, 100, 100, 100, h, w, 1, s1, mean, std, op, None)
    assert call(sq=None) == SAT_ERR_ARG
    assert call(mean=None) == SAT_ERR_ARG
    assert call(std=None) == SAT_ERR_ARG
    assert call(h=101) == SAT_ERR_WINDOW
    assert call(op=96) == SAT_ERR_ARG
    assert call(mean=OUT) == SAT_ERR_ARG                             # outputs overlap
    assert call(std=SQ + 8) == SAT_ERR_ARG                           # output overlaps a table


def test_multi_and_batch_validation(lib):
    hs = (ctypes.c_int64 * 2)(10, 20)
    ws = (ctypes.c_int64 * 2)(10, 200)
    outs = (ctypes.c_void_p * 2)(OUT, OUT2)
    pitches = (ctypes.c_int64 * 2)(200, 200)
    assert lib.window_sum_multi(SAT, SAT_U8, 100, 120, 120, 2, hs, ws, 1, outs, SAT_U32, pitches, None) == SAT_ERR_WINDOW
    assert lib.window_sum_multi(SAT, SAT_U8, 100, 120, 120, 0, hs, ws, 1, outs, SAT_U32, pitches, None) == SAT_ERR_ARG
    assert lib.window_sum_multi(SAT, SAT_U8, 100, 120, 120, 9, hs, ws, 1, outs, SAT_U32, pitches, None) == SAT_ERR_ARG
    items = (BatchItem * 2)()
    for i in range(2):
        items[i].image, items[i].H, items[i].W, items[i].image_pitch = IMG + i * 0x1000000, 50, 60, 60
        items[i].sat, items[i].sat_pitch = SAT + i * 0x1000000, 60
    need = lib.sat_batch_workspace_bytes(items, 2, SAT_U8, 0)
    assert need > 256
    assert lib.sat_build_batched(items, 0, SAT_U8, WS, need, None) == SAT_ERR_ARG
    assert lib.sat_build_batched(items, 2, SAT_U8, WS, need - 1, None) == SAT_ERR_WORKSPACE
    items[1].sat = items[0].sat + 8                                  # tables of two items overlap
    assert lib.sat_build_batched(items, 2, SAT_U8, WS, need, None) == SAT_ERR_ARG
    items[1].sat = SAT + 0x1000000
    items[1].sat_sq = SQ                                             # mixed squared / not squared
    assert lib.sat_build_batched(items, 2, SAT_U8, WS, need, None) == SAT_ERR_ARG
    items[1].sat_sq = None
    items[1].W = 0
    assert lib.sat_build_batched(items, 2, SAT_U8, WS, need, None) == SAT_ERR_ARG
    assert b"item 1" in lib.sat_last_error()


def test_fused_build_stats_validation(lib):
    """sat_build_stats_batched: every build and statistics argument error, before any HIP call."""
    items = (BatchItem * 2)()
    for i in range(2):
        o = i * 0x1000000
        items[i].image, items[i].H, items[i].W, items[i].image_pitch = IMG + o, 50, 60, 64
        items[i].sat, items[i].sat_sq, items[i].sat_pitch = SAT + o, SQ + o, 64
        items[i].sum_out, items[i].mean_out, items[i].std_out, items[i].out_pitch = OUT + o, OUT2 + o, OUT3 + o, 64
    need = lib.sat_build_stats_workspace_bytes(items, 2, SAT_U16)
    assert need > lib.sat_batch_workspace_bytes(items, 2, SAT_U16, 1)
    assert lib.sat_build_stats_workspace_bytes(items, 0, SAT_U16) == 0

    def call(n=2, ptype=SAT_U16, h=8, w=8, s=2, ws=WS, wsb=None):
        return lib.sat_build_stats_batched(items, n, ptype, h, w, s, ws, need if wsb is None else wsb, None)
    assert call(n=0) == SAT_ERR_ARG
    assert call(ptype=SAT_U32) == SAT_ERR_ARG
    assert call(wsb=need - 1) == SAT_ERR_WORKSPACE
    assert call(ws=None) == SAT_ERR_WORKSPACE
    assert call(ws=WS + 16) == SAT_ERR_ARG                           # not 256-byte aligned
    assert call(h=51) == SAT_ERR_WINDOW
    assert call(s=0) == SAT_ERR_ARG
    items[1].mean_out = 0
    assert call() == SAT_ERR_ARG
    items[1].mean_out = OUT2 + 0x1000000
    items[1].std_out = items[0].std_out                              # outputs of two items overlap
    assert call() == SAT_ERR_ARG
    items[1].std_out = OUT3 + 0x1000000
    items[0].sum_out = SQ + 0x1000000 + 8                            # an output overlaps a table
    assert call() == SAT_ERR_ARG
    items[0].sum_out = OUT
    items[1].sat_sq = 0                                              # squares needed on every item
    assert call() == SAT_ERR_ARG
    items[0].sat_sq = 0
    assert call() == SAT_ERR_ARG
    assert b"sat_sq" in lib.sat_last_error()


def test_batched_mean_std_workspace_keeps_the_control_header(lib):
    """window_mean_std_batched puts its descriptor table after the 256-byte control header (whose
    fault word sat_workspace_check reads), so it needs 256 bytes more than the table itself; the
    batch workspace size covers both calls."""
    n = 3
    items = (BatchItem * n)()
    for i in range(n):
        b = 0x100000000 * (i + 1)
        items[i].image, items[i].H, items[i].W, items[i].image_pitch = IMG + b, 100, 120, 128
        items[i].sat, items[i].sat_sq, items[i].sat_pitch = SAT + b, SQ + b, 128
        items[i].mean_out, items[i].std_out, items[i].out_pitch = OUT + b, OUT2 + b, 64
    table = (n * 128 + 255) // 256 * 256                            # 128-byte descriptors
    assert lib.window_mean_std_batched(items, n, 8, 8, 2, WS, table, None) == SAT_ERR_WORKSPACE
    assert lib.window_mean_std_batched(items, n, 8, 8, 2, WS, 256 + table - 1, None) == SAT_ERR_WORKSPACE
    assert lib.sat_batch_workspace_bytes(items, n, SAT_U16, 1) >= 256 + 256 * n
    assert lib.window_mean_std_batched(items, n, 8, 8, 2, WS + 8, 4096, None) == SAT_ERR_ARG   # alignment


def test_variants(lib):
    nb, ng = lib.sat_variant_count(0), lib.sat_variant_count(1)
    assert nb >= 5 and ng >= 3
    names = [lib.sat_variant_name(0, i).decode() for i in range(nb)]
    assert any("lookback" in n for n in names) and any("reduce_scan" in n for n in names)
    assert lib.sat_force_variant(0, nb) == SAT_ERR_ARG
    assert lib.sat_force_variant(2, 0) == SAT_ERR_ARG
    assert lib.sat_force_variant(0, 1) == SAT_OK
    assert lib.sat_force_variant(0, -1) == SAT_OK


def test_variant_supported(lib):
    nb, ng = lib.sat_variant_count(0), lib.sat_variant_count(1)
    names = [lib.sat_variant_name(0, i).decode() for i in range(nb)]
    for i in range(nb):
        assert lib.sat_variant_supported(0, i, SAT_U8, 0) == 1          # every variant builds 8-bit tables
    px8 = names.index("helper_nt_px8_rw12_nw4")
    # two 48-row tiles of 16-bit pixels, four waves' 64-bit squared column sums: beyond 160 KiB of LDS
    assert lib.sat_variant_supported(0, px8, SAT_U16, 1) == 0
    assert lib.sat_variant_supported(0, px8, SAT_U16, 0) == 1
    assert lib.sat_variant_supported(0, px8, SAT_U8, 1) == 1
    assert all(lib.sat_variant_supported(1, i, SAT_U16, 1) == 1 for i in range(ng))
    assert lib.sat_variant_supported(0, nb, SAT_U8, 0) == 0
    assert lib.sat_variant_supported(0, -1, SAT_U8, 0) == 0
    assert lib.sat_variant_supported(2, 0, SAT_U8, 0) == 0
    assert lib.sat_variant_supported(0, 0, SAT_U32, 0) == 0
    # a build forced to a variant without an instantiation for the pixel type is refused
    assert lib.sat_force_variant(0, px8) == SAT_OK
    try:
        ws = lib.sat_build_workspace_bytes(64, 64, SAT_U16, 1)
        st = lib.sat_build(IMG, SAT_U16, 64, 64, 64, SAT, SQ, 64, WS, ws, None)
        assert st == SAT_ERR_ARG and b"does not fit the LDS" in lib.sat_last_error()
    finally:
        lib.sat_force_variant(0, -1)


def test_powers_and_moments_validation(lib):
    P = ctypes.c_void_p
    T3 = (P * 3)(SAT, SQ, OUT)
    ws = lib.sat_powers_workspace_bytes(64, 64, SAT_U8, 3)
    assert ws > 0
    assert lib.sat_powers_workspace_bytes(64, 64, SAT_U8, 5) == 0
    assert lib.sat_powers_workspace_bytes(64, 64, SAT_U32, 2) == 0
    assert lib.sat_powers_workspace_bytes(0, 64, SAT_U8, 2) == 0
    # k beyond 4, a NULL table, overlapping tables, a short workspace
    assert lib.sat_build_powers(IMG, SAT_U8, 64, 64, 64, 5, T3, 64, WS, ws, None) == SAT_ERR_ARG
    assert lib.sat_build_powers(IMG, SAT_U8, 64, 64, 64, 3, (P * 3)(SAT, None, OUT), 64, WS, ws, None) == SAT_ERR_ARG
    assert lib.sat_build_powers(IMG, SAT_U8, 64, 64, 64, 3, (P * 3)(SAT, SAT + 8, OUT), 64, WS, ws, None) == SAT_ERR_ARG
    assert lib.sat_build_powers(IMG, SAT_U8, 64, 64, 64, 3, T3, 64, WS, ws - 8, None) == SAT_ERR_WORKSPACE
    assert lib.sat_build_powers(IMG, SAT_U8, 64, 64, 64, 3, None, 64, WS, ws, None) == SAT_ERR_ARG
    # 62-bit column totals: 16-bit pixel^4 never fits, pixel^3 up to 16384 rows
    T4 = (P * 4)(SAT, SQ, OUT, OUT2)
    ws16 = lib.sat_powers_workspace_bytes(64, 64, SAT_U16, 4)
    assert lib.sat_build_powers(IMG, SAT_U16, 64, 64, 64, 4, T4, 64, WS, ws16, None) == SAT_ERR_OVERFLOW
    big = lib.sat_powers_workspace_bytes(16385, 64, SAT_U16, 3)
    assert lib.sat_build_powers(IMG, SAT_U16, 16385, 64, 64, 3, T3, 64, WS, big, None) == SAT_ERR_OVERFLOW
    # no output, too few tables for the highest statistic, window too large
    assert lib.window_moments(T3, 3, SAT_U8, 64, 64, 64, 8, 8, 1, None, None, None, None, 64, None) == SAT_ERR_ARG
    assert lib.window_moments(T3, 3, SAT_U8, 64, 64, 64, 8, 8, 1, None, None, None, OUT3, 64, None) == SAT_ERR_ARG
    assert lib.window_moments(T3, 3, SAT_U8, 64, 64, 64, 65, 8, 1, OUT2, None, None, None, 64, None) == SAT_ERR_WINDOW
    # outputs overlapping each other or a table
    assert lib.window_moments(T3, 3, SAT_U8, 64, 64, 64, 8, 8, 1, OUT2, OUT2 + 8, None, None, 64, None) == SAT_ERR_ARG
    assert lib.window_moments(T3, 3, SAT_U8, 64, 64, 64, 8, 8, 1, SAT + 8, None, None, None, 64, None) == SAT_ERR_ARG
    # 16-bit skewness: window sums of pixel^3 exceed 64 bits beyond 65536 pixels
    big16 = (P * 3)(SAT, SQ, OUT)
    assert lib.window_moments(big16, 3, SAT_U16, 4096, 4096, 4096, 256, 257, 1, None, None, OUT2, None, 4096,
                              None) == SAT_ERR_OVERFLOW


CARRY, CARRY_SQ, TOT, TOT_SQ = (0x10000000000 * k for k in range(8, 12))


def band(lib, image=IMG, ptype=SAT_U8, H=64, W=80, ipitch=80, carry=CARRY, carry_sq=None, rows_above=100,
         sat=SAT, sat_sq=None, spitch=80, total=TOT, total_sq=None, ws=WS, wsb=None):
    if wsb is None:
        wsb = lib.sat_build_workspace_bytes(H, W, ptype if ptype in (SAT_U8, SAT_U16) else SAT_U8, int(bool(sat_sq)))
    return lib.sat_build_band(image, ptype, H, W, ipitch, carry, carry_sq, rows_above, sat, sat_sq, spitch, total,
                              total_sq, ws, wsb, None)


def test_band_build_validation(lib):
    # everything sat_build checks
    assert band(lib, image=None) == SAT_ERR_ARG
    assert band(lib, ipitch=79) == SAT_ERR_ARG
    assert band(lib, ws=None) == SAT_ERR_WORKSPACE
    # rows above need a carry; a negative count is refused
    assert band(lib, carry=None, rows_above=5) == SAT_ERR_ARG
    assert band(lib, rows_above=-1) == SAT_ERR_ARG
    # squares: a carry needs carry_sq, carry_sq needs sat_sq and a carry, total_sq needs sat_sq
    assert band(lib, sat_sq=SQ) == SAT_ERR_ARG
    assert band(lib, carry_sq=CARRY_SQ) == SAT_ERR_ARG
    assert band(lib, carry=None, rows_above=0, carry_sq=CARRY_SQ, sat_sq=SQ) == SAT_ERR_ARG
    assert band(lib, total_sq=TOT_SQ) == SAT_ERR_ARG
    # totals must not overlap the image, a table or each other; carries must not overlap a table
    assert band(lib, total=SAT + 8) == SAT_ERR_ARG
    assert band(lib, total=IMG + 8) == SAT_ERR_ARG
    assert band(lib, sat_sq=SQ, carry_sq=CARRY_SQ, total_sq=TOT + 16) == SAT_ERR_ARG
    assert band(lib, carry=SAT + 8) == SAT_ERR_ARG
    # a carry equals its total (in place) or overlaps no total
    assert band(lib, carry=TOT + 8) == SAT_ERR_ARG
    # alignment of carries and totals
    assert band(lib, carry=CARRY + 4) == SAT_ERR_ARG
    assert band(lib, total=TOT + 4) == SAT_ERR_ARG
    # workspace must not overlap a carry or a total
    assert band(lib, ws=CARRY) == SAT_ERR_ARG
    assert band(lib, ws=TOT) == SAT_ERR_ARG
    # the 62-bit bound counts the rows above: 16-bit squares, H + rows_above rows
    lim = (1 << 62) // (65535 * 65535)
    assert band(lib, ptype=SAT_U16, H=10, W=1, ipitch=1, spitch=1, sat_sq=SQ, carry_sq=CARRY_SQ,
                rows_above=lim - 5, wsb=1 << 40) == SAT_ERR_OVERFLOW
    # rows above are a row count like any height (at most 2^31 - 1); below that only 16-bit
    # squares can reach 2^62
    assert band(lib, rows_above=1 << 31, wsb=1 << 40) == SAT_ERR_ARG


def test_column_totals_validation(lib):
    def tot(image=IMG, ptype=SAT_U8, H=64, W=80, ipitch=80, carry=None, carry_sq=None, out=TOT, out_sq=None):
        return lib.sat_column_totals(image, ptype, H, W, ipitch, carry, carry_sq, out, out_sq, None)

    assert tot(image=None) == SAT_ERR_ARG
    assert tot(out=None) == SAT_ERR_ARG
    assert tot(ptype=SAT_U32) == SAT_ERR_ARG
    assert tot(H=0) == SAT_ERR_ARG
    assert tot(ipitch=79) == SAT_ERR_ARG
    assert tot(carry_sq=CARRY_SQ) == SAT_ERR_ARG                    # carry_sq without out_sq
    assert tot(carry=CARRY, out_sq=TOT_SQ) == SAT_ERR_ARG            # squares with a carry need carry_sq
    assert tot(out=IMG + 8) == SAT_ERR_ARG                           # output overlaps the image
    assert tot(out_sq=TOT + 8) == SAT_ERR_ARG                        # outputs overlap
    assert tot(carry=TOT + 8) == SAT_ERR_ARG                         # partial overlap of a carry
    assert tot(out=TOT + 4) == SAT_ERR_ARG                           # misaligned


def test_sat_upload_validation(lib):
    """Argument checks that need no device: NULL pointers, an empty copy, misalignment."""
    assert lib.sat_upload(None, OUT, 64, None) == SAT_ERR_ARG
    assert lib.sat_upload(IMG, None, 64, None) == SAT_ERR_ARG
    assert lib.sat_upload(IMG, OUT, 0, None) == SAT_ERR_ARG
    assert lib.sat_upload(IMG + 8, OUT, 64, None) == SAT_ERR_ARG
    assert lib.sat_upload(IMG, OUT + 4, 64, None) == SAT_ERR_ARG
    assert "aligned" in lib.sat_last_error().decode()


def test_force_segments_validation(lib):
    assert lib.sat_force_variant(4, 9) == SAT_ERR_ARG
    assert lib.sat_force_variant(4, -1) == SAT_ERR_ARG
    assert lib.sat_force_variant(4, 3) == SAT_OK
    assert lib.sat_force_variant(4, 0) == SAT_OK


def test_workspace_reserves_the_segment_area(lib):
    """Images of at most 32768 rows get room for the column-segment pre-pass after the lookback
    state; taller ones do not."""
    small = lib.sat_build_workspace_bytes(8192, 8192, SAT_U16, 1)
    assert small >= 256 + 7 * (2 * 8192 + 1) * 8 * 2
    tall_a = lib.sat_build_workspace_bytes(32769, 1000, SAT_U8, 0)
    tall_b = lib.sat_build_workspace_bytes(32768, 1000, SAT_U8, 0)
    assert tall_b - tall_a > 7 * (2 * 32768 + 1) * 8 - 64 * 1024

"""The C boundary without a GPU: header, exported symbols, argument checks."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frnn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(frnn_\w+)\s*\(", text)))


def test_header_compiles_as_c_and_cxx(tmp_path):
    src = tmp_path / "use.c"
    src.write_text('#include "frnn.h"\nint main(void) { frnn_config c = {{0, 0, 0, 0}, 0, 0, 0, 0}; frnn_stats s; (void)c; (void)s; return FRNN_OK; }\n')
    for std, lang in (("-std=c99", "c"), ("-std=c++17", "c++")):
        subprocess.run(["gcc" if lang == "c" else "g++", std, "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-fsyntax-only", "-x", lang, f"-I{os.path.dirname(HEADER)}", str(src)], check=True)


@pytest.fixture(scope="module")
def lib():
    from paper_2202_06929_amd import frnn
    if not os.path.exists(frnn.LIB_PATH):
        pytest.fail("libfrnn.so is not built: run __graft_entry__.build()")
    return frnn.lib()


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert {"frnn_build", "frnn_workspace_bytes", "frnn_status_string"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2202_06929_amd", "libfrnn.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (frnn_\w+)", out))
    assert set(names) <= exported


def test_status_strings(lib):
    from paper_2202_06929_amd import frnn
    for st in range(7):
        assert frnn.status_string(st) != "unknown status"
    assert frnn.status_string(99) == "unknown status"


def test_workspace_bytes_is_monotone_and_rejects_bad_sizes(lib):
    from paper_2202_06929_amd import frnn
    a = frnn.workspace_bytes(1000, 8)
    assert a > 0
    assert frnn.workspace_bytes(2000, 8) > a
    assert frnn.workspace_bytes(1000, 12) > a
    for n, d in ((-1, 8), (10, 2), (10, 65), (2 ** 31, 8)):
        assert frnn.workspace_bytes(n, d) == 0


def _call(lib, points=0, n=10, d=8, r=0.1, K=4, ws=0, wsb=0, src=0, dst=0, cap=0, cfg=None, E=True):
    from paper_2202_06929_amd import frnn
    e = ctypes.c_int64(-7)
    st = lib.frnn_build(ctypes.c_void_p(points), n, d, ctypes.c_float(r), K, ctypes.c_void_p(ws), wsb,
                        ctypes.c_void_p(src), ctypes.c_void_p(dst), cap,
                        ctypes.byref(e) if E else None,
                        ctypes.byref(cfg) if cfg is not None else None, None, None)
    return st, e.value


def test_argument_errors_return_before_touching_a_device(lib):
    from paper_2202_06929_amd import frnn
    ERR = frnn.FRNN_ERR_ARG
    assert _call(lib, n=-1)[0] == ERR
    assert _call(lib, d=2)[0] == ERR
    assert _call(lib, d=65)[0] == ERR
    for r in (0.0, -0.5, float("nan"), float("inf")):
        assert _call(lib, r=r)[0] == ERR
    assert _call(lib, K=0)[0] == ERR
    assert _call(lib, K=frnn.MAX_K + 1)[0] == ERR
    assert _call(lib, cap=-1)[0] == ERR
    assert _call(lib, E=False)[0] == ERR
    assert _call(lib, n=10)[0] == ERR            # null points / workspace
    bad = frnn.FrnnConfig()
    bad.dims[0], bad.dims[1], bad.dims[2] = 0, 1, 1
    assert _call(lib, cfg=bad)[0] == ERR
    bad.dims[0], bad.dims[1], bad.dims[2] = 0, 1, 8
    assert _call(lib, cfg=bad)[0] == ERR
    bad = frnn.FrnnConfig()
    bad.cell_div = 4
    assert _call(lib, cfg=bad)[0] == ERR
    for axes in (1, 2, 5, -1):
        bad = frnn.FrnnConfig()
        bad.axes = axes
        assert _call(lib, cfg=bad)[0] == ERR
    bad = frnn.FrnnConfig()
    bad.axes, bad.cell_div = 4, 2                 # four binned coordinates need cell_div 1
    assert _call(lib, cfg=bad)[0] == ERR
    bad = frnn.FrnnConfig()
    bad.axes = 4
    assert _call(lib, d=3, cfg=bad)[0] == ERR    # more binned coordinates than d
    bad.dims[0], bad.dims[1], bad.dims[2], bad.dims[3] = 0, 1, 2, 1
    assert _call(lib, cfg=bad)[0] == ERR         # repeated coordinate
    bad.dims[3] = 8
    assert _call(lib, cfg=bad)[0] == ERR         # coordinate out of range
    bad = frnn.FrnnConfig()
    bad.grid_mult = 3
    assert _call(lib, cfg=bad)[0] == ERR
    assert _call(lib, n=2 ** 31)[0] == frnn.FRNN_ERR_UNSUPPORTED
    # n = 0 succeeds with no edges and no device work.
    assert _call(lib, n=0) == (frnn.FRNN_OK, 0)
    # A workspace smaller than required is reported before any launch.
    assert _call(lib, points=0x1000, ws=0x100000, wsb=16)[0] == frnn.FRNN_ERR_WORKSPACE
    # A workspace that is not 256-byte aligned is refused.
    assert _call(lib, points=0x1000, ws=0x100010, wsb=1 << 40)[0] == ERR


def _noalloc_call(lib, points=0, n=10, d=8, r=0.1, K=4, src=0, dst=0, cap=0, cfg=None, E=True):
    e = ctypes.c_int64(-7)
    st = lib.frnn_build_noalloc(ctypes.c_void_p(points), n, d, ctypes.c_float(r), K, ctypes.c_void_p(src),
                                ctypes.c_void_p(dst), cap, ctypes.byref(e) if E else None,
                                ctypes.byref(cfg) if cfg is not None else None, None, None)
    return st, e.value


def test_noalloc_checks_return_before_touching_a_device(lib):
    from paper_2202_06929_amd import frnn
    ERR = frnn.FRNN_ERR_ARG
    assert _noalloc_call(lib, n=-1)[0] == ERR
    assert _noalloc_call(lib, d=2)[0] == ERR
    assert _noalloc_call(lib, K=0)[0] == ERR
    assert _noalloc_call(lib, E=False)[0] == ERR
    assert _noalloc_call(lib, n=10)[0] == ERR           # null points
    assert _noalloc_call(lib, points=0x1000, cap=8)[0] == ERR  # null outputs with room for edges
    timing = frnn.FrnnConfig()
    timing.flags = frnn.FLAG_TIMING
    assert _noalloc_call(lib, points=0x1000, cfg=timing)[0] == ERR
    assert _noalloc_call(lib, n=2 ** 31)[0] == frnn.FRNN_ERR_UNSUPPORTED
    assert _noalloc_call(lib, n=0) == (frnn.FRNN_OK, 0)
    # Sizes beyond the library's fixed array are refused on the host.
    limit = frnn.NOALLOC_SCRATCH_MIB << 20
    n_fit = 120_000
    assert frnn.workspace_bytes(n_fit, 8) <= limit
    n_big = 1_000_000
    assert frnn.workspace_bytes(n_big, 8) > limit
    assert _noalloc_call(lib, points=0x1000, n=n_big)[0] == frnn.FRNN_ERR_WORKSPACE


def _batch_call(lib, offsets, n_events=None, d=8, r=0.1, K=4, ws=0, wsb=0, cap=0, eo=True):
    import numpy as np
    from paper_2202_06929_amd import frnn
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n_events = off.size - 1 if n_events is None else n_events
    out = np.zeros(max(n_events + 1, 1), dtype=np.int64)
    return lib.frnn_build_batch(ctypes.c_void_p(0), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_events,
                                d, ctypes.c_float(r), K, ctypes.c_void_p(ws), wsb, ctypes.c_void_p(0),
                                ctypes.c_void_p(0), cap,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if eo else None, None, None,
                                None)


def test_batch_argument_errors_and_workspace_sizes(lib):
    from paper_2202_06929_amd import frnn
    ERR = frnn.FRNN_ERR_ARG
    assert _batch_call(lib, [0, 10, 5]) == ERR          # decreasing offsets
    assert _batch_call(lib, [0, 10], n_events=0) == ERR
    assert _batch_call(lib, [0, 10], eo=False) == ERR
    assert _batch_call(lib, [0, 10], d=2) == ERR
    assert _batch_call(lib, [0, 10], K=0) == ERR
    assert _batch_call(lib, [0, 0, 0]) == frnn.FRNN_OK  # no rows: nothing to do
    assert _batch_call(lib, [0, 10, 20]) == ERR         # null points and workspace
    assert _batch_call(lib, [0, 10, 20], ws=0x100000, wsb=16) == ERR  # points still null
    one = frnn.batch_workspace_bytes([0, 1000], 8)
    assert one == frnn.workspace_bytes(1000, 8)
    two = frnn.batch_workspace_bytes([0, 1000, 3000], 8)
    assert two > frnn.batch_workspace_bytes([0, 2000], 8) - 1 > one
    assert frnn.batch_workspace_bytes([0, 5, 3], 8) == 0
    assert frnn.batch_workspace_bytes([0, 2 ** 31], 8) == 0


def test_distance_kernels_use_no_fused_or_packed_float_ops(tmp_path):
    # Every product and sum of the distance is rounded on its own: the search and
    # the placement pass (which collects long lists again) must contain no fused
    # multiply-add and no packed FP32 op.
    from paper_2202_06929_amd import build_lib
    asm = open(build_lib.device_asm(str(tmp_path))).read()
    kernels = re.split(r"\n(?=_ZN\S+:)", asm)
    checked = 0
    for body in kernels:
        name = body.split(":", 1)[0]
        if "k_search" not in name and "k_place" not in name:
            continue
        checked += 1
        body = body.split(".Lfunc_end", 1)[0]
        bad = re.findall(r"\b(v_fma\w*|v_fmac\w*|v_mad_f32\w*|v_mac_f32\w*|v_pk_fma\w*|v_pk_mul_f32|v_pk_add_f32)\b",
                         body)
        assert not bad, f"{name}: {sorted(set(bad))}"
        assert re.search(r"\bv_(sub|subrev)_f32", body) and re.search(r"\bv_mul_f32", body)
    assert checked >= 16 + 8


def test_components_argument_errors_and_workspace_sizes(lib):
    from paper_2202_06929_amd import frnn
    ws = lib.frnn_components_workspace_bytes
    assert ws(-1) == 0 and ws(2 ** 31) == 0
    sizes = [ws(n) for n in (0, 1, 1000, 120_000, 2 ** 31 - 1)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:])) and sizes[0] > 0
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: every check fails first

    def call(src=fake, dst=fake, e=10, n=10, wsp=fake, wsb=1 << 30, labels=fake):
        return lib.frnn_components(src, dst, e, n, None, ctypes.c_float(0.5), wsp, wsb, labels, None, None)

    assert call(e=-1) == frnn.FRNN_ERR_ARG
    assert call(n=-1) == frnn.FRNN_ERR_ARG
    assert call(n=2 ** 31) == frnn.FRNN_ERR_UNSUPPORTED
    assert call(src=None) == frnn.FRNN_ERR_ARG
    assert call(labels=None) == frnn.FRNN_ERR_ARG
    assert call(wsp=None) == frnn.FRNN_ERR_ARG
    assert call(wsp=ctypes.c_void_p((1 << 20) + 8)) == frnn.FRNN_ERR_ARG  # not 256-byte aligned
    assert call(wsb=ws(10) - 1) == frnn.FRNN_ERR_WORKSPACE
    assert lib.frnn_components_async(fake, fake, 10, 10, None, ctypes.c_float(0.5), fake, 1 << 30, fake, None,
                                     None) == frnn.FRNN_ERR_ARG  # no result buffer

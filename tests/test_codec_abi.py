"""CPU tests of libebr's host side: exported symbols, the posting-list codec, input validation.

No GPU is used: the library loads without a device, and these entry points are host-only.
"""
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import paper_2511_22460_amd as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ebr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ebr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = E.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(E.EXPORTS)
    assert "gfx950" in E.version()


# ----------------------------------------------------------------------------- codec

def roundtrip(ids):
    ids = np.asarray(ids, dtype=np.uint32)
    blob = E.codec_encode(ids)
    n = len(ids)
    hdr = 16 * ((n + 63) // 64)
    assert len(blob) >= hdr and (len(blob) - hdr) % 4 == 0
    out = E.codec_decode(blob, n)
    assert out.dtype == np.uint32 and np.array_equal(out, ids)
    return blob


@pytest.mark.parametrize("ids", [
    [], [0], [2**32 - 1], [0, 2**32 - 1], list(range(64)), list(range(65)),
    list(range(1000, 1127)), list(range(5, 5 + 128)), list(range(7, 7 + 129)),
    [0, 1, 2**31, 2**32 - 2, 2**32 - 1], [31, 32, 63, 64, 95, 96],
])
def test_codec_edge_cases(ids):
    roundtrip(ids)


def test_codec_consecutive_ids_cost_only_headers():
    blob = roundtrip(np.arange(10_000, 10_000 + 640))
    assert len(blob) == 10 * 16          # gap width 0: no packed words


def test_codec_gap_width_is_per_chunk():
    rng = np.random.default_rng(1)
    dense = np.sort(rng.choice(100_000, 6400, replace=False))
    sparse = np.sort(rng.choice(2**32 - 1, 6400, replace=False))
    assert len(roundtrip(dense)) < len(roundtrip(sparse)) / 2


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(min_value=0, max_value=2**32 - 1), max_size=400, unique=True))
def test_codec_roundtrip_property(xs):
    roundtrip(sorted(xs))


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2**32 - 1), st.lists(st.integers(0, 5000), max_size=300))
def test_codec_roundtrip_gaps(start, gaps):
    ids, cur = [], start
    for g in gaps:
        if cur > 2**32 - 1:
            break
        ids.append(cur)
        cur += g + 1
    roundtrip(ids)


def test_codec_rejects_bad_input():
    with pytest.raises(E.EbrError) as ei:
        E.codec_encode(np.array([5, 5], np.uint32))
    assert ei.value.status == E.EBR_EINVAL
    with pytest.raises(E.EbrError):
        E.codec_encode(np.array([9, 3], np.uint32))
    blob = bytearray(E.codec_encode(np.arange(0, 300, 3)))
    with pytest.raises(E.EbrError):
        E.codec_decode(bytes(blob[:10]), 100)          # truncated header
    blob[4] = 40                                       # gap width > 32
    with pytest.raises(E.EbrError):
        E.codec_decode(bytes(blob), 100)


# ----------------------------------------------------------------------------- validation

def tiny(n_ads=100, dim=16):
    rng = np.random.default_rng(0)
    E_ = rng.normal(size=(n_ads, dim)).astype(np.float32)
    offs = np.array([0, 3, 3, 6], np.int64)
    ids = np.array([1, 5, 9, 0, 50, 99], np.uint32)
    w = rng.normal(size=6).astype(np.float32)
    return E_, offs, ids, w


def test_index_size_is_exact_and_host_only():
    E_, offs, ids, w = tiny()
    n = E.index_size(E_, offs, ids, w)
    assert n > 0 and n % 256 == 0
    # an ids-only index (no weights, the paper's binary L) drops the weight section: here six
    # FP32 weights, one 256-byte aligned block
    assert E.index_size(E_, offs, ids, None) == n - 256


@pytest.mark.parametrize("mutate, status", [
    (lambda E_, o, i, w: (E_, o, np.array([1, 5, 5, 0, 50, 99], np.uint32), w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_, o, np.array([1, 9, 5, 0, 50, 99], np.uint32), w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_, o, np.array([1, 5, 9, 0, 50, 100], np.uint32), w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_, o, i, np.array([0, 0, np.nan, 0, 0, 0], np.float32)), E.EBR_EINVAL),
    (lambda E_, o, i, w: (np.where(np.arange(E_.size).reshape(E_.shape) == 7, np.inf, E_)
                          .astype(np.float32), o, i, w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_[:, :8].copy(), o, i, w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_, np.array([1, 3, 3, 6], np.int64), i, w), E.EBR_EINVAL),
    (lambda E_, o, i, w: (E_, np.array([0, 3, 2, 6], np.int64), i, w), E.EBR_EINVAL),
])
def test_index_validation_errors(mutate, status):
    args = mutate(*tiny())
    with pytest.raises(E.EbrError) as ei:
        E.index_size(*args)
    assert ei.value.status == status


def test_reduced_precision_copies_grow_the_arena():
    E_, offs, ids, w = tiny(n_ads=1000, dim=64)
    base = E.index_size(E_, offs, ids, w)
    bf = E.index_size(E_, offs, ids, w, dtypes=1 | (1 << E.BF16))
    f8 = E.index_size(E_, offs, ids, w, dtypes=1 | (1 << E.FP8E4M3))
    assert bf - base >= 1024 * 64 * 2 and f8 - base >= 1024 * (64 + 4)
    with pytest.raises(E.EbrError) as ei:
        E.index_size(E_, offs, ids, w, dtypes=1 << 5)
    assert ei.value.status == E.EBR_EINVAL


def test_server_entry_points_reject_null_handles():
    lib = E.load()
    import ctypes
    opts = E.ServerOpts(0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.ebr_server_create(None, None, 0, ctypes.byref(opts), ctypes.byref(h)) == E.EBR_EINVAL
    t = ctypes.c_uint64()
    assert lib.ebr_submit(None, None, None, None, ctypes.byref(t)) == E.EBR_EINVAL
    assert lib.ebr_poll(None, 1, 0) == E.EBR_EINVAL
    assert lib.ebr_server_stats(None, None) == E.EBR_EINVAL
    assert lib.ebr_server_reset_stats(None) == E.EBR_EINVAL
    assert lib.ebr_server_destroy(None) == E.EBR_EINVAL
    assert "NULL" in lib.ebr_last_error().decode()


def test_tuning_and_graph_entry_points_reject_null_handles():
    lib = E.load()
    import ctypes
    sh = E.LaunchShape(0, 0, 0)
    assert lib.ebr_set_launch_shape(None, E.F32, 1, ctypes.byref(sh)) == E.EBR_EINVAL
    assert lib.ebr_get_launch_shape(None, E.F32, 1, ctypes.byref(sh)) == E.EBR_EINVAL
    rep = E.TuneReport()
    assert lib.ebr_autotune(None, None, None, 0, None, None, 0, None, ctypes.byref(rep)) == E.EBR_EINVAL
    assert lib.ebr_score_topk_graph(None, None, None, None, 0, None, None, None) == E.EBR_EINVAL
    assert lib.ebr_graph_stats(None, None) == E.EBR_EINVAL
    assert lib.ebr_graph_create(None) == E.EBR_EINVAL
    lib.ebr_graph_destroy(None)  # a no-op


def test_abi_struct_sizes_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes the C compiler gives include/ebr.h's."""
    import ctypes
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "sizes.c"
    names = ["ebr_launch_shape", "ebr_tune_report", "ebr_graph_info", "ebr_server_opts",
             "ebr_batch", "ebr_query", "ebr_server_info", "ebr_timings", "ebr_build_desc",
             "ebr_index_info"]
    src.write_text('#include <stdio.h>\n#include "ebr.h"\nint main(void) {\n' +
                   "".join(f'  printf("%zu\\n", sizeof({n}));\n' for n in names) +
                   "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    mine = [E.LaunchShape, E.TuneReport, E.GraphInfo, E.ServerOpts, E.Batch, E.Query,
            E.ServerStats, E.Timings, E.BuildDesc, E.IndexInfo]
    assert got == [ctypes.sizeof(t) for t in mine]

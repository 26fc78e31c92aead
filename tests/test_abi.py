"""The C ABI on the CPU: the library loads, exports every function the header
declares, and its host-side argument and graph checks return the documented
codes without touching a GPU."""
import ctypes
import os

import numpy as np
import pytest

from paper_1701_01772_amd import inputs, lge


def _gpu_count():
    try:
        import torch
        return torch.cuda.device_count()
    except Exception:
        return 0


def test_library_exports_every_header_symbol():
    lib = lge.load()
    names = lge.header_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_header_error_codes_match_binding():
    txt = open(lge.HEADER).read()
    for name in ("LGE_OK", "LGE_EINVAL", "LGE_ENOMEM", "LGE_EGRAPH", "LGE_EDEVICE", "LGE_ERANGE",
                 "LGE_EBUSY", "LGE_ETIMEDOUT", "LGE_ECANCELED", "LGE_ENOTFOUND"):
        assert ("#define %s " % name) in txt
        code = getattr(lge, name)
        assert lge.lge_strerror(code) != "unknown error"


def test_struct_sizes_match_header_layout():
    # lge_result: 5 scalars + 4 x 18 u128 + 4 x 18 doubles
    assert ctypes.sizeof(lge.Result) == 8 * 5 + 16 * 18 * 4 + 8 * 18 * 4
    assert ctypes.sizeof(lge.Opts) == 4 * 8


@pytest.mark.parametrize("case,code", [
    (([0, 1, 2], [1, 0]), lge.LGE_OK),                    # one edge
    (([0], []), lge.LGE_OK),                              # empty graph, n = 0
    (([0, 0, 0], []), lge.LGE_OK),                        # isolated vertices
    (([0, 1, 1], [1]), lge.LGE_EGRAPH),                   # asymmetric
    (([0, 2, 3, 4], [1, 2, 0, 0]), lge.LGE_OK),
    (([0, 1, 2], [0, 1]), lge.LGE_EGRAPH),                # self-loops
    (([0, 2, 4], [1, 1, 0, 0]), lge.LGE_EGRAPH),          # duplicate entries
    (([0, 2, 3, 4], [2, 1, 0, 0]), lge.LGE_EGRAPH),       # unsorted row
    (([0, 1, 2], [5, 0]), lge.LGE_EGRAPH),                # id out of range
    (([0, 2, 1], [1, 0]), lge.LGE_EGRAPH),                # decreasing row_ptr
    (([1, 2, 3], [1, 0]), lge.LGE_EGRAPH),                # row_ptr[0] != 0
    (([0, 1, 2, 3], [1, 0, 0]), lge.LGE_EGRAPH),          # odd number of entries
])
def test_validate_csr_host(case, code):
    rp, cl = case
    assert lge.lge_validate_csr_host(np.array(rp), np.array(cl)) == code


def test_validate_csr_host_accepts_generated_graphs():
    for g in (inputs.erdos_renyi(300, 0.05, 1), inputs.chung_lu(2000, 8.0, 2.1, 500.0, 2),
              inputs.rmat(10, 8, 0.57, 0.19, 0.19, 3)):
        assert lge.lge_validate_csr_host(g.row_ptr, g.col) == lge.LGE_OK


def test_bad_probability_rejected_before_any_device_work():
    lib = lge.load()
    r = lge.Result()
    for p in (0.0, -0.5, 1.5, float("nan"), float("inf")):
        assert lib.lge_estimate(None, None, p, 0, None, ctypes.byref(r)) == lge.LGE_EINVAL
        assert lib.lge_estimate_range(None, None, p, 0, 0, 0, None, ctypes.byref(r)) == lge.LGE_EINVAL
        assert lib.lge_autotune(None, None, p, None) == lge.LGE_EINVAL


def test_null_arguments_rejected():
    lib = lge.load()
    r = lge.Result()
    assert lib.lge_estimate(None, None, 0.5, 0, None, ctypes.byref(r)) == lge.LGE_EINVAL
    assert lib.lge_open(0, None) == lge.LGE_EINVAL
    assert lib.lge_close(None) == lge.LGE_EINVAL
    assert lib.lge_graph_destroy(None) == lge.LGE_EINVAL
    assert lib.lge_autotune_reset(None) == lge.LGE_EINVAL
    assert lib.lge_set_build_scratch(None, 0) == lge.LGE_EINVAL
    assert lib.lge_count_batch(None, None, None, None) == lge.LGE_EINVAL
    assert lib.lge_validate_csr_host(-1, None, None) == lge.LGE_EINVAL
    assert lib.lge_graph_n(None) == -1


@pytest.mark.skipif(_gpu_count() > 0, reason="a GPU is present")
def test_open_without_gpu_reports_device_error():
    with pytest.raises(lge.LgeError) as ei:
        lge.lge_open(0)
    assert ei.value.code == lge.LGE_EDEVICE


def test_opts_defaults():
    o = lge.lge_opts_default()
    assert 1 <= o.wave_max_deg <= 512
    assert o.block_max_deg == 1024
    assert o.probe_ratio > 0

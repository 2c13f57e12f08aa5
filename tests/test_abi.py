"""The C ABI without a GPU: the in-tree librqrcp.so loads, exports every
function that include/rqrcp.h declares, and its host-only entry points
(options, status strings, sizing, argument checks) behave as documented.
No kernel is launched here."""
import ctypes
import os
import re

import pytest
import torch

import paper_1505_08115_amd as R
from paper_1505_08115_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rqrcp.h")

ERR_ARG, ERR_UNSUPPORTED = 1, 4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rqrcp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.LIB_PATH):
        build_lib.build()
    return R.load_library()


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for required in ("rqrcp_factor", "rqrcp_factor_sizes", "rqrcp_apply_q", "rqrcp_apply_p", "rqrcp_lowrank",
                     "rqrcp_lowrank_backward", "rqrcp_sketch", "rqrcp_create", "rqrcp_destroy"):
        assert required in names


def test_library_exports_every_declared_function(lib):
    raw = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_exactly_the_header(lib):
    assert sorted(R.EXPORTS) == declared_functions()


def test_default_options_and_status_strings(lib):
    o = R.Opts()
    lib.rqrcp_default_opts(ctypes.byref(o))
    assert (o.block, o.oversample, o.rank, o.pivot, o.precision, o.tail, o.fixed_pivots) == (128, 10, 0, 0, 0, 0, 0)
    assert o.seed == 0 and not o.G and not o.info and o.power == 0 and o.panel_pivot == 0 and o.diagonalize == 0
    for st in range(7):
        assert lib.rqrcp_status_string(st)


def test_factor_sizes_follow_the_block_structure(lib):
    tau, T, S, work = R.factor_sizes(8192, 8192, torch.float64, block=256, oversample=10)
    assert tau == 8192 and T == 32 * 256 * 256 and S == 0
    assert work > 8 * 8192 * 256 * 4          # at least G, V, V^T and V T^T
    # the orthonormal form stores S blocks; a truncated factorization only its blocks
    _, _, S2, _ = R.factor_sizes(1024, 1024, torch.float64, block=128, oversample=8, pivot="ortho")
    assert S2 > 0
    tau3, T3, _, _ = R.factor_sizes(1000, 800, torch.float64, block=64, oversample=8, rank=100)
    assert tau3 == 100 and T3 == 2 * 64 * 64
    # FP32 storage (mixed) needs its own staging
    assert R.factor_sizes(4096, 4096, torch.float32, block=128, oversample=16, precision="mixed")[3] > 0


@pytest.mark.parametrize("m,n,kw,status", [
    (100, 200, {}, ERR_ARG),                                # m < n
    (100, 100, {"block": 0}, ERR_ARG),                      # b < 1
    (100, 100, {"oversample": -1}, ERR_ARG),                # p < 0
    (100, 100, {"rank": 101}, ERR_ARG),                     # k > n
    (2000, 2000, {"block": 600}, ERR_UNSUPPORTED),          # b > 512
    (2000, 2000, {"block": 400, "oversample": 200}, ERR_UNSUPPORTED),   # b + p > 512
    (100, 100, {"power": -1}, ERR_ARG),                     # q < 0
    (100, 100, {"power": 9}, ERR_ARG),                      # q > 8
    (100, 100, {"pivot": "ortho", "panel_pivot": True}, ERR_UNSUPPORTED),  # P-hat: permutation form only
    (100, 100, {"diagonalize": True}, ERR_UNSUPPORTED),     # Section 6.2 blocks: orthonormal pivoting only
    (400, 400, {"pivot": "ortho", "diagonalize": True, "block": 257}, ERR_UNSUPPORTED),  # b <= 256
])
def test_factor_sizes_rejects_invalid_arguments(lib, m, n, kw, status):
    o = R.make_opts(**kw)
    a, b, c, d = (ctypes.c_size_t() for _ in range(4))
    st = lib.rqrcp_factor_sizes(0, m, n, ctypes.byref(o), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                ctypes.byref(d))
    assert st == status
    assert lib.rqrcp_last_error(None)


def test_option_combinations_and_their_workspace(lib):
    a, b, c, d = (ctypes.c_size_t() for _ in range(4))
    args = (ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d))
    # the power iteration and P-hat in both storage types, the mixed mode included
    for dt in (0, 1):
        assert lib.rqrcp_factor_sizes(dt, 500, 400, ctypes.byref(R.make_opts(power=2)), *args) == 0
        assert lib.rqrcp_factor_sizes(dt, 500, 400, ctypes.byref(R.make_opts(panel_pivot=True)), *args) == 0
    assert lib.rqrcp_factor_sizes(1, 500, 400, ctypes.byref(R.make_opts(power=1, precision="mixed")), *args) == 0
    # power steps hold Y X^T: (b + p) m doubles, within the workspace of every storage type
    for dt in (torch.float64, torch.float32):
        _, _, _, w1 = R.factor_sizes(500, 400, dt, power=1)
        assert w1 >= (128 + 10) * 500 * 8
    # diagonalised blocks in either storage type; S grows by U'_i, V'_i (b x b each) per block
    o = R.make_opts(pivot="ortho", diagonalize=True, block=32)
    assert lib.rqrcp_factor_sizes(1, 500, 400, ctypes.byref(o), *args) == 0
    assert lib.rqrcp_factor_sizes(1, 500, 400, ctypes.byref(R.make_opts(diagonalize=True)), *args) == ERR_UNSUPPORTED
    _, _, s0, _ = R.factor_sizes(500, 400, torch.float64, pivot="ortho", block=32)
    _, _, s1, _ = R.factor_sizes(500, 400, torch.float64, pivot="ortho", block=32, diagonalize=True)
    assert s1 - s0 == 2 * 13 * 32 * 32
    # the U'/V' blocks are the last 2 nb b^2 doubles of S
    assert lib.rqrcp_diag_offset(400, 400, 32) == s1 - 2 * 13 * 32 * 32 == s0
    _, _, s2, _ = R.factor_sizes(500, 400, torch.float64, pivot="ortho", block=100, rank=250, diagonalize=True)
    assert lib.rqrcp_diag_offset(400, 250, 100) == s2 - 2 * 3 * 100 * 100
    # fixed pivots draw no sketch: the power setting is ignored
    assert lib.rqrcp_factor_sizes(1, 500, 400, ctypes.byref(R.make_opts(power=1, fixed_pivots=True)), *args) == 0


def test_work_byte_queries_are_host_only_and_positive(lib):
    assert lib.rqrcp_apply_q_work_bytes(0, 4096, 4096, 128, 64) > 0
    assert lib.rqrcp_apply_p_work_bytes(0, 64, 4096, 4096, 128) > 0
    assert lib.rqrcp_lowrank_work_bytes(0, 4096, 4096, 256, 128) > 0
    assert lib.rqrcp_lowrank_backward_work_bytes(0, 4096, 4096, 256, 128) > 0
    assert lib.rqrcp_lowrank_work_bytes(0, 0, 4096, 256, 128) == 0     # invalid sizes report 0


def test_colmajor_always_copies():
    a = torch.randn(5, 3, dtype=torch.float64)
    c = R.colmajor(a)
    c2 = R.colmajor(c)                     # already column-major: still a new tensor
    assert c.stride(0) == 1 and c2.stride(0) == 1
    assert c2.data_ptr() != c.data_ptr() and torch.equal(c2, a)

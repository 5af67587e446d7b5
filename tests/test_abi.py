"""The C-ABI library loads and exports every entry point its header declares;
host-only entry points (parameters, workspace sizes, status strings) work
without a GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hgp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hgp_status|const char \*)\s*(hgp_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def H():
    import paper_2303_17679_amd as H
    if not os.path.exists(H.LIB_PATH):
        from paper_2303_17679_amd import build
        build.build()
    H.lib()
    return H


def test_header_symbols_exported(H):
    names = declared()
    assert len(names) == 30
    assert names == sorted(H.EXPORTS)
    L = ctypes.CDLL(H.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_timing_sample_arguments(H):
    # host state only: the sampling period and phase are checked, nothing runs
    L = H.lib()
    assert L.hgp_timing_sample(0, 0) == -1
    assert L.hgp_timing_sample(3, 3) == -1
    assert L.hgp_timing_sample(3, 2) == 0
    assert L.hgp_timing_sample(1, 0) == 0


def test_status_strings(H):
    L = H.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.hgp_status_str(s)
    assert L.hgp_status_str(0) == b"ok"


def test_default_params(H):
    p = H.Params()
    assert H.lib().hgp_default_params(64, ctypes.byref(p)) == 0
    assert (p.k, p.eps_num, p.eps_den, p.limit_factor, p.coarsen_subrounds, p.lp_subrounds, p.lp_rounds) == \
        (64, 3, 100, 160, 3, 5, 5)


def test_workspace_sizes_host_only(H):
    prm = H.params(64)
    for op in (H.OP_COARSEN, H.OP_CONTRACT, H.OP_REFINE, H.OP_PARTITION, H.OP_VALIDATE, H.OP_INITIAL):
        a = H.workspace_bytes(op, 1000, 1000, 5000, prm)
        b = H.workspace_bytes(op, 100000, 100000, 500000, prm)
        assert 0 < a <= b
    # partition needs at least every single step
    n, m, p = 4096000, 4096000, 28518400
    part = H.workspace_bytes(H.OP_PARTITION, n, m, p, prm)
    for op in (H.OP_COARSEN, H.OP_CONTRACT, H.OP_REFINE):
        assert part > H.workspace_bytes(op, n, m, p, prm)


def test_bad_parameters_rejected_on_host(H):
    out = ctypes.c_size_t(0)
    L = H.lib()
    assert L.hgp_workspace_bytes(H.OP_REFINE, 10, 10, 10, ctypes.byref(H.params(1)), ctypes.byref(out)) == -1
    assert L.hgp_workspace_bytes(H.OP_REFINE, 10, 10, 10, ctypes.byref(H.params(257)), ctypes.byref(out)) == -5
    assert L.hgp_workspace_bytes(H.OP_REFINE, 10, 10, 10, ctypes.byref(H.params(4, eps=(1, 0))),
                                 ctypes.byref(out)) == -1
    assert L.hgp_workspace_bytes(99, 10, 10, 10, None, ctypes.byref(out)) == -1
    assert L.hgp_workspace_bytes(H.OP_REFINE, 10, 10, 10, ctypes.byref(H.params(4, ip=2)), ctypes.byref(out)) == -1
    assert L.hgp_rb_initial_partition(None, ctypes.byref(H.params(4)), None, None, 0, None) == -1
    # null hypergraph / workspace pointers are refused before any device work
    assert L.hgp_partition(None, ctypes.byref(H.params(4)), None, None, None, None, 0, None) == -1
    assert L.hgp_coarsen(None, None, 0, None, None, None, 0, None) == -1


def test_rb_workspace_covers_a_bisection_and_the_path(H):
    # recursive bipartitioning needs a whole k = 2 multilevel workspace plus
    # the subhypergraphs along the recursion; the partition with ip = 1 adds it
    n, m, p = 100000, 120000, 600000
    bis = H.workspace_bytes(H.OP_PARTITION, n, m, p, H.params(2))
    for k in (2, 3, 8, 64, 256):
        rb = H.workspace_bytes(H.OP_RB, n, m, p, H.params(k))
        assert rb > bis
        assert H.workspace_bytes(H.OP_PARTITION, n, m, p, H.params(k, ip=1)) > \
            H.workspace_bytes(H.OP_PARTITION, n, m, p, H.params(k)) + bis
    assert H.workspace_bytes(H.OP_RB, n, m, p, H.params(256)) > H.workspace_bytes(H.OP_RB, n, m, p, H.params(8))


def test_static_refine_rejects_levels_beyond_its_scratch(H):
    # rejected on the host from the sizes alone, before any device work
    import ctypes
    L = H.lib()
    s = H._HG(1 << 24, 1 << 24, 1 << 26, None, None, None, None, None, None)
    prm = H.params(64)
    part = ctypes.c_uint32(0)
    st = L.hgp_refine_lp_static(ctypes.byref(s), ctypes.byref(prm), 0, ctypes.addressof(part), None, None, None)
    assert st == -3  # HGP_E_WORKSPACE
    need = ctypes.c_size_t(0)
    assert L.hgp_workspace_bytes(3, 1 << 24, 1 << 24, 1 << 26, ctypes.byref(prm), ctypes.byref(need)) == 0
    assert need.value > H.STATIC_SCRATCH_BYTES

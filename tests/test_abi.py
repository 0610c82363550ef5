"""The C-ABI library loads and exports every symbol the header declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "pfmf.h")).read()
    return sorted(set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = header_symbols()
    for name in ["pf_setup_mesh", "pf_apply_residual", "pf_apply_jacobian", "pf_apply_adjoint", "pf_pmg_vcycle"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2607_21150_amd import pfmf
    if not os.path.exists(pfmf.LIB_PATH):
        pytest.fail("libpfmf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(pfmf.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name
    assert set(header_symbols()) == set(pfmf.EXPORTED)


def test_null_context_is_rejected_without_gpu():
    from paper_2607_21150_amd import pfmf
    L = pfmf.load()
    assert L.pf_sizes(None, None, None, None) == pfmf.PF_EINVAL
    assert b"null" in L.pf_last_error()
    rc = L.pf_setup_mesh(None, None, 0, None, None, None, None, None, None)
    assert rc == pfmf.PF_EINVAL


def test_branch_calls_reject_a_null_context_without_gpu():
    from paper_2607_21150_amd import pfmf
    L = pfmf.load()
    assert L.pf_set_branches(None, None, 0, None) == pfmf.PF_EINVAL
    assert L.pf_commit_state_branches(None, None, None, None, None) == pfmf.PF_EINVAL


def test_geometry_call_rejects_a_null_context_without_gpu():
    from paper_2607_21150_amd import pfmf
    L = pfmf.load()
    assert L.pf_set_geometry(None, None, None) == pfmf.PF_EINVAL


def test_table_setup_rejects_null_arguments_without_gpu():
    from paper_2607_21150_amd import pfmf
    L = pfmf.load()
    assert L.pf_setup_mesh_table(None, None, None, None, 0, None, None, None, None, None, None) == pfmf.PF_EINVAL
    out = ctypes.c_void_p()
    md = pfmf.TableMeshDesc(3, 0, 0)
    assert L.pf_setup_mesh_table(ctypes.byref(md), None, None, None, 0, None, None, None, None, None,
                                 ctypes.byref(out)) == pfmf.PF_EINVAL
    assert not out.value

"""The C-ABI library loads and exports every entry point the header
declares (no compute calls: runs without a GPU)."""
import os
import re

import pytest

from paper_2202_12309_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pkh_[a-z_0-9]+)\s*\(", txt, re.M)
    return names


def test_header_declares_the_boundary():
    names = set(_declared())
    for must in ["pkh_mesh_create", "pkh_mesh_destroy", "pkh_mesh_blocks", "pkh_state_upload",
                 "pkh_state_download", "pkh_exchange_boundaries", "pkh_step", "pkh_get_time",
                 "pkh_set_time", "pkh_set_refinement_flags", "pkh_regrid", "pkh_conserved_totals",
                 "pkh_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libpkhydro.so is not built (run __graft_entry__.build())")
    L = binding.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(_declared()) <= set(binding._SIGS)


def test_last_error_callable_without_gpu():
    assert binding.lib().pkh_last_error() is not None

"""CPU checks of the C ABI library: it loads, exports every function the
header declares, validates arguments without touching a device, and the
host-side interface numbering agrees with the oracle's."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2211_14969_amd import hps
from paper_2211_14969_amd import harness
from oracle import interface as itf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hps.LIB_PATH):
        from paper_2211_14969_amd import build
        build.build()
    return hps.load()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hps_leaf_build", "hps_leaf_condense", "hps_leaf_recover"):
        assert n in names
    assert set(names) == set(hps.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(0, -7, -1):
        s = hps.status_string(code)
        assert s and s != "unknown status"
    assert hps.status_string(42) == "unknown status"


def test_argument_validation_without_device(lib):
    vp = ctypes.c_void_p
    out = vp()
    desc = (hps.hps_leaf_desc * 1)()
    assert lib.hps_leaf_build(None, desc, 1, ctypes.byref(out)) == hps.HPS_ERR_INVALID
    assert lib.hps_ctx_create(None, None) == hps.HPS_ERR_INVALID
    assert lib.hps_leaf_condense(None, 0, 0.0, 0, None, None, None, None, 0) == hps.HPS_ERR_INVALID
    assert lib.hps_leaf_recover(None, None, None, None, 0) == hps.HPS_ERR_INVALID
    assert lib.hps_batch_export(None, None, None) == hps.HPS_ERR_INVALID
    assert lib.hps_batch_group_dims(None, 0, None, None, None, None) == hps.HPS_ERR_INVALID
    assert lib.hps_batch_nleaf(None) == -1
    assert lib.hps_batch_destroy(None) == hps.HPS_OK
    assert lib.hps_leaf_condense_noalloc(None, 0, 0.0, 0, None, None, None, None, 0) == \
        hps.HPS_ERR_INVALID
    assert lib.hps_batch_redo_flags(None, None) == hps.HPS_ERR_INVALID
    assert lib.hps_batch_lanes(None) == -1


@pytest.mark.parametrize("nx,ny,p", [(4, 4, 8), (3, 2, 5), (1, 1, 6), (5, 3, 12)])
def test_host_edge_numbering_matches_oracle(nx, ny, p):
    ids, dmask = harness.edge_ids(nx, ny, p)
    num = itf.numbering(nx, ny, p)
    np.testing.assert_array_equal(ids, num.slot)
    np.testing.assert_array_equal(dmask, num.dirichlet)


def test_python_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(hps, "_lib", None)
    with pytest.raises(RuntimeError):
        hps.load(str(tmp_path / "missing.so"))

"""The C-ABI library loads and exports every entry point declared in
include/*.h (no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "claire.h")
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(claire_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("claire_transport", "claire_gradient", "claire_hessian_matvec",
                     "claire_solve", "claire_ctx_create", "claire_last_error",
                     "claire_net_create", "claire_net_train_step", "claire_net_warm_start"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2401_17493_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libclaire_gfx950.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_struct_layouts_match_header():
    from paper_2401_17493_amd import _lib
    text = open(HEADER).read()
    for cname, pystruct in (("claire_opts", _lib.ClaireOpts), ("claire_stats", _lib.ClaireStats)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"([A-Za-z_0-9]+)\s*(?:,|;)", body)
        assert fields == [f for f, _ in pystruct._fields_], (cname, fields)


def test_library_refuses_to_load_when_missing(monkeypatch):
    from paper_2401_17493_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libclaire_gfx950.so")
    with pytest.raises(RuntimeError):
        _lib.load()


def test_binding_imports_without_gpu():
    # the torch binding must import (and stay syntactically valid) on the CPU
    from paper_2401_17493_amd import claire, warmstart
    assert claire.FIELD_GRAD_STATE == 3 and claire.KERNEL_COPY == 3
    assert hasattr(claire.Context, "time_kernel")
    assert hasattr(warmstart.Net, "train_step") and hasattr(warmstart, "resample")

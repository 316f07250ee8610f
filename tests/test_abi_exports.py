"""The C-ABI library loads without a GPU and exports every entry point that the
public header declares; the Python binding names each of them.  No compute call is
made here."""
import ctypes
import os
import re

import gpu_setup

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "af.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:af_status|void|const char\s*\*)\s*(af_[a-z0-9_]+)\s*\(", text, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared()
    for core in ("af_create", "af_destroy", "af_last_error", "af_set_geometry", "af_set_lens",
                 "af_set_slowness", "af_beamform", "af_loss_and_grad", "af_autofocus_step"):
        assert core in names, core
    assert len(names) >= 24


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gpu_setup.ensure_built())
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"declared in af.h but not exported: {missing}"


def test_binding_names_every_entry_point():
    src = open(os.path.join(ROOT, "paper_2608_06853_amd", "_lib.py")).read()
    missing = [n for n in declared() if n not in src]
    assert not missing, f"no binding for: {missing}"


def test_kernel_family_names_follow_the_header():
    """The binding's per-family timing names are in the order of the header's
    AF_K_ ids, one per id."""
    from paper_2608_06853_amd import _lib
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    ids = {k: int(v) for k, v in re.findall(r"\b(AF_K_[A-Z_]+)\s*=\s*(\d+)", text)}
    count = ids.pop("AF_K_COUNT")
    assert sorted(ids.values()) == list(range(count))
    assert len(_lib.KERNELS) == count
    for name, i in ids.items():
        short = name[len("AF_K_"):].lower()
        assert _lib.KERNELS[i].replace("_grid", "").replace("grad_", "") == short, (name, _lib.KERNELS[i])

"""The C-ABI library loads, exports every symbol its header declares, and its host-only
entry points (sizes, validation) behave as documented. No GPU compute here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_12739_amd import binding as b
from synth import ModelConfig, blob_size

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "conet.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(conet_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = b.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(b.EXPORTS)


@pytest.mark.parametrize("K,L,C,Ci,m", [(2, 2, 32, 8, 2), (3, 4, 64, 16, 4), (4, 6, 96, 32, 8), (1, 1, 16, 8, 1)])
def test_weight_count_matches_blob_layout(K, L, C, Ci, m):
    for dt in ("f32", "bf16"):
        cfg = b.make_config(K, L, C, Ci, m, dt)
        assert b.weight_count(cfg) == blob_size(ModelConfig(K, L, C, Ci, m))
        assert b.workspace_bytes(cfg) > 0
        # BatchNorm after the fusion: the blob ends with a running mean and variance per block
        bn = b.make_config(K, L, C, Ci, m, dt, norm="bn")
        assert b.weight_count(bn) == blob_size(ModelConfig(K, L, C, Ci, m)) + 2 * L * C


def test_workspace_grows_with_max_res():
    small = b.workspace_bytes(b.make_config(3, 4, 64, 16, 4, "bf16", max_res=1000))
    big = b.workspace_bytes(b.make_config(3, 4, 64, 16, 4, "bf16", max_res=100000))
    assert big - small >= 99000 * 64 * 2 * 9 * 0.99   # 3K activation buffers of C bf16 channels


@pytest.mark.parametrize("kw,msg", [
    (dict(K=9, L=2, C=32, C_in=8, m=2), "branches"),
    (dict(K=2, L=2, C=48, C_in=8, m=2), "no kernel"),
    (dict(K=2, L=2, C=32, C_in=8, m=9), "bits_per_symbol"),
    (dict(K=2, L=2, C=32, C_in=8, m=2, fuse_mask=0b100), "fuse_mask"),
    (dict(K=2, L=2, C=16, C_in=16, m=2, norm="bn", train=True), "BatchNorm"),
])
def test_invalid_configs_are_rejected_with_a_message(kw, msg):
    lib = b.load()
    cfg = b.make_config(kw.pop("K"), kw.pop("L"), kw.pop("C"), kw.pop("C_in"), kw.pop("m"), "bf16", **kw)
    assert b.weight_count(cfg) == 0
    assert msg in lib.conet_last_error().decode()


def test_create_rejects_bad_arguments_without_touching_the_gpu():
    lib = b.load()
    cfg = b.make_config(2, 2, 32, 8, 2, "f32")
    h = ctypes.c_void_p()
    n = b.weight_count(cfg)
    w = np.zeros(n, np.float32)
    fp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert lib.conet_create(ctypes.byref(cfg), fp, n - 1, ctypes.c_void_p(256), 1 << 30, ctypes.byref(h)) == 1
    assert "blob" in lib.conet_last_error().decode()
    assert lib.conet_create(ctypes.byref(cfg), fp, n, None, 1 << 30, ctypes.byref(h)) == 1
    assert lib.conet_create(ctypes.byref(cfg), fp, n, ctypes.c_void_p(257), 1 << 30, ctypes.byref(h)) == 1
    assert "aligned" in lib.conet_last_error().decode()
    assert lib.conet_create(ctypes.byref(cfg), fp, n, ctypes.c_void_p(256), 16, ctypes.byref(h)) == 3
    assert lib.conet_forward(None, None, 1, 14, 8, None, 0, None) == 1
    assert lib.conet_destroy(None) == 1


def _header_struct_fields(name):
    """Field names, in order, of `typedef struct { ... } name;` in include/conet.h."""
    src = open(os.path.join(os.path.dirname(__file__), "..", "include", "conet.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1] if not decl.startswith("const ") else decl.split(None, 2)[2]
        fields += [n.strip().lstrip("*") for n in names.split(",")]
    return fields


@pytest.mark.parametrize("struct", ["conet_config", "conet_request", "conet_serve_stats"])
def test_binding_structs_match_the_header(struct):
    """The ctypes mirrors of the C structs list the header's fields in the header's order."""
    assert [f for f, _ in getattr(b, struct)._fields_] == _header_struct_fields(struct)

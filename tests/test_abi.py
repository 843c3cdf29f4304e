"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/bmlp.h, and its host-only helpers behave (no GPU work)."""
import ctypes
import os
import re

import pytest

from paper_2408_10369_amd import build as pkg_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmlp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bmlp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2408_10369_amd as P
    if not os.path.exists(P.LIB_PATH):
        pkg_build.build()
    return P.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "bmlp_rms" in names and "bmlp_smp" in names and "bmlp_compose_linear" in names
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_header():
    import paper_2408_10369_amd as P
    assert sorted(P.EXPORTS) == _declared()


def test_opts_defaults_and_struct_sizes(L):
    import paper_2408_10369_amd as P
    o = P.make_opts()
    assert o.size == ctypes.sizeof(P.Opts) == 40
    assert o.dispatch == P.DISPATCH_PLAIN and o.product_arm == P.ARM_AUTO and o.rms_variant == 0
    # ... mfma_ops_issued, then gathers (int32, padded to 8), gather_ms, gather_bytes
    assert ctypes.sizeof(P.Stats) == 4 + 4 + 256 + 4 + 4 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert L.bmlp_version() >= 100


def test_null_handle_is_einval(L):
    import paper_2408_10369_amd as P
    rc = L.bmlp_rms(None, None, None, 0, 0, None, None, None)
    assert rc == P.EINVAL
    assert b"null handle" in L.bmlp_last_error()
    assert L.bmlp_destroy(None) == P.OK


def test_create_without_device_fails_cleanly(L):
    import paper_2408_10369_amd as P
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = L.bmlp_create(ctypes.byref(h), 0)
    assert rc in (P.EDEVICE, P.EINVAL)
    assert not h.value


def test_tune_buckets_host_only(L):
    """Buckets of the autotuned tile code: 4 sizes by the dense operation count, 4 operand classes."""
    import paper_2408_10369_amd as P
    C = P.Context
    assert C.tune_candidates(P.TUNE_MFMA_PRODUCT) >= 2 and C.tune_candidates(P.TUNE_VALU_PRODUCT) >= 2
    assert C.tune_candidates(7) == 0 and C.tune_buckets(7) == 0
    assert C.tune_buckets(P.TUNE_MFMA_PRODUCT) == 16
    k = P.TUNE_MFMA_PRODUCT
    assert C.tune_bucket_of(k, 2048, 2048, 2048) == 4 * 0 + 2          # unknown density counts as dense
    assert C.tune_bucket_of(k, 4096, 4096, 4096, 1e-5) == 4 * 1 + 0
    assert C.tune_bucket_of(k, 8192, 8192, 8192, 1e-3) == 4 * 2 + 1
    assert C.tune_bucket_of(k, 16384, 16384, 16384, 0.3) == 4 * 3 + 2
    assert C.tune_bucket_of(k, 16384, 16384, 16384, 0.3, structured=True) == 4 * 3 + 3
    assert C.tune_bucket_of(k, 65536, 65536, 65536, -1.0) == 4 * 3 + 2
    assert C.tune_bucket_of(k, -1, 1, 1) == -1 and C.tune_bucket_of(9, 1, 1, 1) == -1

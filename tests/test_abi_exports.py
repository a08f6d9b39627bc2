"""The C-ABI library loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("hpt_create", "hpt_scene_upload", "hpt_cache_build", "hpt_trace_submit",
              "hpt_field_read", "hpt_job_wait"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_14173_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.skip("libhpt.so not built")
    lib = ctypes.CDLL(_binding.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert sorted(_binding.SIGNATURES) == _declared()


def test_no_device_fails_loudly():
    """Without a gfx950 device the library refuses to create a context
    (there is no CPU fallback)."""
    import paper_2606_14173_amd as hpt
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(hpt.HptError) as e:
        hpt.Context(0)
    assert e.value.name in ("HPT_ENODEV",)


def test_version_string():
    import paper_2606_14173_amd as hpt
    assert b"gfx950" in hpt.load().hpt_version()

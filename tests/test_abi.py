"""The C ABI without a GPU: libat.so loads, exports every entry point that
include/at.h declares, and the binding refuses a library built from other sources.
No compute call is made here."""
import os
import re

import pytest

from paper_2204_01133_amd import binding
from paper_2204_01133_amd import build as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "at.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(at_\w+)\s*\(", text, flags=re.M)))


def test_header_declarations_found():
    names = declared_functions()
    assert "at_init" in names and "at_batch_step" in names and "at_free" in names
    assert sorted(binding.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    L = binding.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_stale_library_refused(monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(B, "source_hash", lambda: "0000000000000000")
    with pytest.raises(RuntimeError, match="not built from the current sources"):
        binding.load_library()

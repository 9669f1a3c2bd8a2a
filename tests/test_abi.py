"""The C-ABI library loads and exports every entry point include/*.h declares
(no compute: these run without a GPU)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names.update(re.findall(r"\b(mra_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mra_build_tree", "mra_loglik", "mra_predict", "mra_free_tree", "mra_last_error", "mra_tree_info"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1905_00141_amd import mra
    for n in _declared():
        assert hasattr(mra._lib, n), n
    assert sorted(mra.EXPORTED) == sorted(_declared())


def test_no_device_is_reported_not_hidden():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1905_00141_amd import mra
    with pytest.raises(mra.MraError) as e:
        mra.Tree(np.array([0.1]), np.array([0.2]), np.array([1.0]), J=4, r=4, M=2)
    assert e.value.code == mra.MRA_EDEVICE

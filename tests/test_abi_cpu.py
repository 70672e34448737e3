"""The C-ABI library loads and exports every symbol include/deconv.h declares;
host-side argument checks (no GPU compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "deconv.h")
LIB = os.path.join(ROOT, "paper_1602_01410_amd", "libdeconv.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(deconv_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("deconv_plan_create", "deconv_admm_run", "deconv_admm_backward", "deconv_plan_destroy"):
        assert n in names


def test_library_exports_all_declared_symbols():
    if not os.path.exists(LIB):
        pytest.skip("libdeconv.so not built")
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_export_list_matches_header():
    from paper_1602_01410_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_host_argument_checks():
    if not os.path.exists(LIB):
        pytest.skip("libdeconv.so not built")
    from paper_1602_01410_amd import binding
    L = binding.lib()
    assert L.deconv_status_str(0) == b"ok"
    assert binding.workspace_size([dict(height=64, width=64, ksize=5)]) > 64 * 64 * 40
    bad = [([dict(height=100, width=64, ksize=5)], {}, 2),       # 100 = 2^2 5^2
           ([dict(height=64, width=64, ksize=4)], {}, 2),        # even kernel
           ([dict(height=8, width=8, ksize=9)], {}, 2),          # kernel too large
           ([dict(height=64, width=64, ksize=5, mask_kind=7)], {}, 1),
           ([dict(height=64, width=64, ksize=5)], dict(alpha=2.5), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=0), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=10, tol_primal=1e-3), 1),
           ([dict(height=4096, width=64, ksize=5)], {}, 2)]
    for images, opts, code in bad:
        with pytest.raises(binding.DeconvError) as e:
            binding.workspace_size(images, **opts)
        assert e.value.code == code, (images, opts)
    # checkpoints grow the workspace
    a = binding.workspace_size([dict(height=64, width=64, ksize=5)])
    b = binding.workspace_size([dict(height=64, width=64, ksize=5)], ckpt_every=5, max_iters=20)
    assert b > a

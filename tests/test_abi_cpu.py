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
           ([dict(height=4096, width=64, ksize=5)], {}, 2),
           ([dict(height=64, width=64, ksize=5)], dict(bgs_passes=-1), 1),
           ([dict(height=64, width=64, ksize=5)], dict(bgs_passes=65), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=10, bgs_passes=0), 1),
           ([dict(height=64, width=64, ksize=5)], dict(separable_blur=2), 1),
           ([dict(height=64, width=64, ksize=5)], dict(adapt_t=-1.0), 1),
           ([dict(height=64, width=64, ksize=5)], dict(warm_iters=-1), 1),
           ([dict(height=64, width=64, ksize=5)], dict(warm_iters=10, warm_tau=0.0), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=10, bgs_passes=2), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=10, adapt_t=3.0), 1),
           ([dict(height=64, width=64, ksize=5)], dict(ckpt_every=5, max_iters=10, warm_iters=5), 1),
           ([dict(height=64, width=64, ksize=5)], dict(spectra_hint=3), 1),
           ([dict(height=64, width=64, ksize=5)], dict(row_tiles=3), 1),
           ([dict(height=64, width=64, ksize=5)], dict(row_threads=256), 1),
           ([dict(height=64, width=64, ksize=5)], dict(col_threads=1024), 1),
           ([dict(height=64, width=64, ksize=5)], dict(small_images=3), 1),
           ([], {}, 1)]                                            # empty batch
    for images, opts, code in bad:
        with pytest.raises(binding.DeconvError) as e:
            binding.workspace_size(images, **opts)
        assert e.value.code == code, (images, opts)
    # per-image pass counts (0) are accepted
    assert binding.workspace_size([dict(height=64, width=64, ksize=5)], bgs_passes=0) > 0
    # checkpoints grow the workspace
    a = binding.workspace_size([dict(height=64, width=64, ksize=5)])
    b = binding.workspace_size([dict(height=64, width=64, ksize=5)], ckpt_every=5, max_iters=20)
    assert b > a


def test_binding_struct_layout_matches_header(tmp_path):
    """Sizes and field offsets of the option and statistics structs as the C
    compiler lays them out, against the ctypes mirrors of the binding."""
    import subprocess
    from paper_1602_01410_amd import binding
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "deconv.h"', 'int main(void) {']
    for cname, cls in (("deconv_options", binding.Options), ("deconv_stats", binding.Stats),
                       ("deconv_image_desc", binding.ImageDesc)):
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append('return 0; }')
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, cls in (("deconv_options", binding.Options), ("deconv_stats", binding.Stats),
                       ("deconv_image_desc", binding.ImageDesc)):
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_option_defaults_match_header():
    """deconv_options_default fills the defaults the header documents."""
    if not os.path.exists(LIB):
        pytest.skip("libdeconv.so not built")
    from paper_1602_01410_amd import binding
    o = binding.default_options()
    assert o.alpha == 2.0
    assert (o.check_every, o.use_graph, o.batched, o.ckpt_every, o.profile, o.schedule) == (0, 1, 1, 0, 0, 0)
    assert (o.tol_primal, o.tol_dual, o.adapt_t) == (0.0, 0.0, 0.0)
    assert (o.bgs_passes, o.warm_iters, o.channels, o.spectra_hint) == (1, 0, 1, 0)
    assert abs(o.warm_tau - 1e-3) < 1e-9
    assert (o.row_tiles, o.row_threads, o.col_threads, o.small_images, o.separable_blur) == (0, 0, 0, 2, 1)
    assert not o.tune_cache

"""libaf.so loads without a GPU, exports every function include/af.h declares,
and the binding's ctypes structures have the header's layout (CPU only; no
compute call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "af.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libaf():
    from paper_2608_06412_amd import af
    if not os.path.exists(af.LIB_PATH):
        from paper_2608_06412_amd import build
        build.build()
    return af.load_library()


def test_exports_every_declared_symbol(libaf):
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(libaf, n), n
    from paper_2608_06412_amd import af
    assert set(af.SIGNATURES) == set(names)


def test_struct_layouts_match_header(tmp_path):
    from paper_2608_06412_amd import af
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "af.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(af_config),'
                   ' sizeof(af_tool), sizeof(af_frame_stats), sizeof(af_score_stats),'
                   ' offsetof(af_config, hbm_budget), offsetof(af_config, max_blocks));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).split()))
    exp = [ctypes.sizeof(af.Config), ctypes.sizeof(af.Tool), ctypes.sizeof(af.FrameStats),
           ctypes.sizeof(af.ScoreStats), af.Config.hbm_budget.offset, af.Config.max_blocks.offset]
    assert got == exp


def test_config_default_and_argument_errors(libaf):
    """Host-side argument checks need no GPU."""
    from paper_2608_06412_amd import af
    cfg = af.Config()
    assert libaf.af_config_default(ctypes.byref(cfg), 0.01, 0.04) == af.AF_OK
    assert (cfg.n_c, cfg.weight_cap, cfg.conf_min_w, cfg.n_vp, cfg.knn_k) == (5, 2000, 2, 8, 10)
    assert abs(cfg.cos_normal - 0.3420201433256687) < 1e-16
    assert libaf.af_config_default(ctypes.byref(cfg), 0.0, 0.0) == af.AF_EINVAL
    h = ctypes.c_void_p()
    bad = af.Config()
    libaf.af_config_default(ctypes.byref(bad), 0.01, 0.5)   # tau = 50 voxels: too wide
    assert libaf.af_create(ctypes.byref(bad), ctypes.byref(h)) == af.AF_EINVAL
    bad2 = af.Config()
    libaf.af_config_default(ctypes.byref(bad2), 0.01, 0.04)
    bad2.n_vp = 9
    assert libaf.af_create(ctypes.byref(bad2), ctypes.byref(h)) == af.AF_EINVAL
    assert not h.value


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU and says so (before touching any device)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout

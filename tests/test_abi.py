"""The C-ABI library loads without a GPU and exports every function that
include/art.h declares (no compute calls)."""
import ctypes
import os
import subprocess

import pytest

from paper_2103_07417_amd import art

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    names = art.header_functions()
    assert {"art_render", "art_render_uniform", "art_trace_points", "art_metrics",
            "art_image_size", "art_last_error", "art_release"} <= set(names)
    L = art.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", art.LIB_PATH]).decode()
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for n in names:
        assert n in exported, n


def test_image_size_and_validation_host_only():
    cfg = dict(a=0.94, r_cam=1000.0, inc_deg=163.0, fov=40.0, nx0=129, ny0=129, levels=3,
               model="thermal", nstokes=4)
    assert art.image_size(cfg) == (1025, 1025)
    cfg2 = dict(cfg, nx0=65, ny0=33, levels=6)
    assert art.image_size(cfg2) == (4097, 2049)
    with pytest.raises(art.ArtError):
        art.image_size(dict(cfg, nx0=1))
    with pytest.raises(art.ArtError):
        art.image_size(dict(cfg, levels=21))
    with pytest.raises(art.ArtError):          # 2^32 pixels
        art.image_size(dict(cfg, nx0=65537, ny0=65537, levels=0))


def test_last_error_is_a_message():
    try:
        art.image_size(dict(a=0.0, r_cam=1000.0, inc_deg=60.0, fov=40.0, nx0=1, levels=0,
                            model="toy_disk"))
    except art.ArtError as e:
        assert "base grid" in str(e)
    assert isinstance(art.lib().art_last_error(), bytes)


def test_product_package_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2103_07417_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "ray_oracle" not in txt, f

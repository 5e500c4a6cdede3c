"""CPU checks of the C ABI: the header compiles as C, the built library
exports every declared call, the binding exposes the same names, and
argument validation fails cleanly before any GPU work is queued."""
import ctypes
import os
import subprocess

import pytest

from _helpers import HEADER, LIB, ensure_built, header_functions

import synth


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    return ctypes.CDLL(LIB)


def test_headers_are_plain_c():
    import glob, os
    for h in sorted(glob.glob(os.path.join(os.path.dirname(HEADER), "*.h"))):
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", h])


def test_every_declared_call_is_exported(lib):
    names = header_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], stdout=subprocess.PIPE, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in names:
        assert n in exported, n
        getattr(lib, n)
    # internal launchers stay hidden
    assert not any("launch_fp" in e for e in exported)


def test_binding_names_match_header(lib):
    from paper_1402_4381_amd import lalm
    for n in header_functions():
        assert hasattr(lalm, n), n
    assert set(lalm.EXPORTS) == set(header_functions())


def _geom(**kw):
    from paper_1402_4381_amd import lalm
    g = synth.geometry_of(synth.get_config("fan2d_128"))
    g.update(kw)
    return lalm._geometry(g)


@pytest.mark.parametrize("kw,M", [
    (dict(nx=0), 4),
    (dict(dsd=500.0), 4),            # dsd <= dso
    (dict(dso=60.0, dsd=120.0), 4),  # source inside the image's circumscribed circle
    (dict(detector=1), 4),
    (dict(nz=2), 4),                 # 2D needs nz = 1
    (dict(n_rows=3), 4),
    ({}, 0),
    ({}, 181),                       # more subsets than views
    (dict(dx=-1.0), 4),
    (dict(kind=7), 4),
    (dict(n_bins=(1 << 20) + 1, ds=1e-4), 4),                 # beyond the 24-bit row offsets
    (dict(kind=1, nz=8, n_rows=257, dt=0.01), 4),             # more than 256 detector rows
    (dict(kind=1, nz=8, n_rows=256, dt=0.01, n_bins=1 << 20, ds=1e-4, n_views=16, n_views_per_turn=16), 4),
])                                                            # ^ a 4 GiB subset sinogram
def test_invalid_geometry_rejected_before_gpu_work(lib, kw, M):
    from paper_1402_4381_amd import lalm
    h = ctypes.c_void_p()
    st = lalm._lib.lalm_plan_geometry(ctypes.byref(_geom(**kw)), M, 1, ctypes.byref(h))
    assert st == lalm.LALM_E_INVALID
    assert h.value is None
    assert len(lalm.lalm_last_error()) > 0


@pytest.mark.parametrize("batch", [0, -1, 65536])
def test_invalid_batch_rejected(lib, batch):
    from paper_1402_4381_amd import lalm
    h = ctypes.c_void_p()
    assert lalm._lib.lalm_plan_geometry(ctypes.byref(_geom()), 4, batch, ctypes.byref(h)) == lalm.LALM_E_INVALID
    assert h.value is None and "batch" in lalm.lalm_last_error()


def test_null_arguments_rejected(lib):
    from paper_1402_4381_amd import lalm
    L = lalm._lib
    assert L.lalm_plan_geometry(None, 4, 1, None) == lalm.LALM_E_INVALID
    assert L.lalm_plan_info(None, None, None, None, None, None, None) == lalm.LALM_E_INVALID
    assert L.lalm_project_subset(None, 0, None, None, None, None, None) == lalm.LALM_E_INVALID
    assert L.lalm_backproject_subset(None, 0, None, None, 1.0, 0, None) == lalm.LALM_E_INVALID
    assert L.lalm_sqs_denom(None, None, None, None) == lalm.LALM_E_INVALID
    assert L.lalm_iterate(None, None, None, 1, None, None, None) == lalm.LALM_E_INVALID
    assert L.lalm_dot_f64(None, None, None, 0, None, None) == lalm.LALM_E_INVALID
    assert L.lalm_plan_destroy(None) == lalm.LALM_E_INVALID
    assert lalm.lalm_version().startswith("lalm")
    assert L.lalm_unet_create(0, 16, 16, None) == lalm.LALM_E_INVALID
    h = ctypes.c_void_p()
    assert L.lalm_unet_create(1, 18, 16, ctypes.byref(h)) == lalm.LALM_E_INVALID   # not a multiple of 4
    from oracle import unet as U
    assert lalm.lalm_unet_param_count() == U.param_count()


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets of the C struct it
    stands for (gcc compiles a probe against the header)."""
    from paper_1402_4381_amd import lalm
    mirrors = {"lalm_geometry": lalm.Geometry, "lalm_problem": lalm.Problem, "lalm_state": lalm.State,
               "lalm_options": lalm.Options, "lalm_stats": lalm.Stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lalm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0; }"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, check=True).stdout.split("\n")
    got = {}
    for l in out:
        if l:
            k1, k2, v = l.split()
            got[(k1, k2)] = int(v)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)

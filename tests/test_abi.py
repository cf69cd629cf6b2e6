"""The C ABI on the CPU: the library loads, exports every function that
include/mcx.h declares, and rejects invalid input before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1711_03244_amd import mcx, nn, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="mcx.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["mcx_create", "mcx_run", "mcx_run_range", "mcx_fluence", "mcx_detected",
              "mcx_stats", "mcx_destroy", "mcx_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = mcx.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(mcx.EXPORTS)
    for n in declared_functions("mcx_nn.h"):
        assert hasattr(lib, n), n
    assert set(declared_functions("mcx_nn.h")) == set(nn.EXPORTS)


def test_default_options():
    o = mcx.mcx_default_options()
    assert o.rr_threshold == pytest.approx(1e-4) and o.rr_m == 10.0
    assert o.n_outside == 1.0 and o.max_detected == 1 << 20 and o.reflect == 0


STRUCTS = ["mcx_medium", "mcx_volume", "mcx_source", "mcx_detector", "mcx_gates",
           "mcx_options", "mcx_run_stats", "mcx_sim", "mcx_tune_result", "mcx_detpost"]


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets the
    C compiler gives the struct of include/mcx.h (compiled here with gcc)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(ROOT, "include")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mcx.h"', "int main(void) {"]
    for name in STRUCTS:
        st = getattr(mcx, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for name in STRUCTS:
        st = getattr(mcx, name)
        assert int(got[f"{name} size"]) == C.sizeof(st), name
        for field, _ in st._fields_:
            assert int(got[f"{name} {field}"]) == getattr(st, field).offset, (name, field)


@pytest.mark.parametrize("bad", [dict(ndet=0), dict(ndet=5000), dict(npath=0), dict(npath=256),
                                 dict(dt_ns=0.0), dict(dt_ns=float("nan")),
                                 dict(t0_ns=float("inf")), dict(ngates=0), dict(ngates=8191)])
def test_detpost_spec_checked_before_the_gpu(bad):
    """Every invalid post-processing spec is refused before any HIP call
    (the record and output pointers are never touched)."""
    spec = dict(ndet=4, npath=2, t0_ns=0.0, dt_ns=0.1, ngates=50, nphoton=1000)
    spec.update(bad)
    sp = mcx.mcx_detpost(spec["ndet"], spec["npath"], spec["t0_ns"], spec["dt_ns"],
                         spec["ngates"], spec["nphoton"])
    st = mcx.lib().mcx_detpost_device(None, 0, C.byref(sp), None, None, None, None)
    assert st == mcx.MCX_EINVAL, mcx.mcx_last_error()
    st = mcx.lib().mcx_detpost_device(None, 10, C.byref(sp), None, None, None, None)
    assert st == mcx.MCX_EINVAL
    assert mcx.lib().mcx_detpost_device(None, 0, None, None, None, None, None) == mcx.MCX_EINVAL
    for fn in (mcx.lib().mcx_detpost_device_noalloc,):
        assert fn(None, 0, C.byref(sp), None, None, None, None) == mcx.MCX_EINVAL
        assert fn(None, 10, C.byref(sp), None, None, None, None) == mcx.MCX_EINVAL
        assert fn(None, 0, None, None, None, None, None) == mcx.MCX_EINVAL
    out = (C.c_double * 8)()
    assert mcx.lib().mcx_detected_process(None, 0, None, out, 8, None, 0) == mcx.MCX_EINVAL


BAD = {
    "source outside grid": dict(src_pos=(70.0, 1.0, 1.0)),
    "direction not unit": dict(src_dir=(0.0, 0.0, 0.9)),
    "zero gates": dict(ngates=0),
    "negative dt": dict(dt=-1.0),
    "roulette M": dict(rr_m=1.0),
    "n outside < 1": dict(n_out=0.5),
}


@pytest.mark.parametrize("case", sorted(BAD))
def test_invalid_problem_rejected(case):
    kw = dict(src_pos=(3.5, 3.5, 0.0))
    kw.update(BAD[case])
    p = W.cube_homogeneous(n=8).replace(**kw)
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_create(p)
    assert e.value.status == mcx.MCX_EINVAL
    assert mcx.mcx_last_error()


def test_invalid_media_rejected():
    p = W.cube_homogeneous(n=8).replace(src_pos=(3.5, 3.5, 0.0))
    for row in [(-0.1, 1.0, 0.0, 1.37), (0.1, 1.0, 1.5, 1.37), (0.1, 1.0, 0.0, 0.9),
                (float("nan"), 1.0, 0.0, 1.37)]:
        with pytest.raises(mcx.McxError) as e:
            mcx.mcx_create(W.with_medium(p, 1, row))
        assert e.value.status == mcx.MCX_EINVAL


def test_label_out_of_range_and_source_in_air_rejected():
    p = W.cube_homogeneous(n=8).replace(src_pos=(3.5, 3.5, 0.0))
    lab = p.labels.copy()
    lab[4, 4, 4] = 7
    with pytest.raises(mcx.McxError):
        mcx.mcx_create(p.replace(labels=lab))
    lab = p.labels.copy()
    lab[0, 3, 3] = 0
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_create(p.replace(labels=lab))
    assert "label 0" in str(e.value)


def test_bad_detector_rejected():
    p = W.cube_sphere(n=20)
    d = p.detectors.copy()
    d[1, 3] = 0.0
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_create(p.replace(detectors=d))
    assert e.value.status == mcx.MCX_EINVAL


def test_bad_launch_options_rejected():
    p = W.cube_homogeneous(n=8).replace(src_pos=(3.5, 3.5, 0.0))
    for kw in [dict(block_size=100), dict(block_size=2048), dict(refill_chunk=5),
               dict(max_events=0), dict(lds_window_cells=36865), dict(kernel_variant=3),
               dict(kernel_variant=-1), dict(kernel_variant=2, accurate_math=1),
               dict(kernel_variant=1, ndigest=10)]:
        with pytest.raises(mcx.McxError) as e:
            mcx.mcx_create(p, **kw)
        assert e.value.status == mcx.MCX_EINVAL


def test_no_device_reported_without_gpu():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    p = W.cube_homogeneous(n=8).replace(src_pos=(3.5, 3.5, 0.0))
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_create(p)
    assert e.value.status == mcx.MCX_ENODEV


def test_null_context_calls_fail_cleanly():
    lib = mcx.lib()
    assert lib.mcx_run(None, 10, 1) == mcx.MCX_EINVAL
    assert lib.mcx_sync(None) == mcx.MCX_EINVAL
    assert lib.mcx_ncells(None) == 0
    assert lib.mcx_set_map_adds(None, mcx.MAP_ADDS_32) == mcx.MCX_EINVAL
    assert lib.mcx_set_launch(None, 0, 0, 0) == mcx.MCX_EINVAL
    lib.mcx_destroy(None)


def test_denoiser_arguments_checked_before_the_gpu():
    L = nn.lib()
    out = C.c_void_p()
    ch = (C.c_int32 * 3)(8, 16, 32)
    assert L.mcx_nn_create(ch, 0, 16, 16, 16, 0, C.byref(out)) == mcx.MCX_EINVAL
    assert L.mcx_nn_create(ch, 3, 16, 16, 10, 0, C.byref(out)) == mcx.MCX_EINVAL  # not a multiple of 4
    assert "multiples of 4" in mcx.mcx_last_error()
    bad = (C.c_int32 * 3)(8, 0, 32)
    assert L.mcx_nn_create(bad, 3, 16, 16, 16, 0, C.byref(out)) == mcx.MCX_EINVAL
    assert L.mcx_nn_layer_forward(7, 4, 4, 4, 1, 1, None, None, None, None, 0, 0, None,
                                  None) == mcx.MCX_EINVAL
    assert L.mcx_nn_layer_forward(nn.MCX_NN_DOWN, 3, 4, 4, 1, 1, None, None, None, None, 0, 0,
                                  None, None) == mcx.MCX_EINVAL
    assert "even" in mcx.mcx_last_error()
    assert L.mcx_nn_param_count(None) == 0
    assert L.mcx_nn_set_fused_backward(None, 1, None) == mcx.MCX_EINVAL
    # augmentation op (fake addresses: the checks run before any HIP call)
    a, b = C.c_void_p(4096), C.c_void_p(8192)
    assert L.mcx_nn_mirror_xy(a, a, 4, 4, 4, 1, None) == mcx.MCX_EINVAL
    assert L.mcx_nn_mirror_xy(None, b, 4, 4, 4, 1, None) == mcx.MCX_EINVAL
    assert L.mcx_nn_mirror_xy(a, b, 4, 4, 4, 8, None) == mcx.MCX_EINVAL
    assert L.mcx_nn_mirror_xy(a, b, 4, 4, 0, 1, None) == mcx.MCX_EINVAL
    assert L.mcx_nn_mirror_xy(a, b, 4, 5, 4, 4, None) == mcx.MCX_EINVAL
    assert "nx == ny" in mcx.mcx_last_error()
    step = C.c_int32()
    assert L.mcx_nn_get_adam(None, a, b, 4, C.byref(step)) == mcx.MCX_EINVAL
    assert L.mcx_nn_get_adam(a, None, b, 4, C.byref(step)) == mcx.MCX_EINVAL
    assert L.mcx_nn_set_adam(a, a, None, 4, 0) == mcx.MCX_EINVAL
    assert L.mcx_nn_set_adam(a, a, b, 4, -1) == mcx.MCX_EINVAL


def test_denoiser_reports_no_device_without_gpu():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    out = C.c_void_p()
    ch = (C.c_int32 * 2)(8, 16)
    assert nn.lib().mcx_nn_create(ch, 2, 8, 8, 8, 0, C.byref(out)) == mcx.MCX_ENODEV


def test_binding_fails_loudly_without_the_library(tmp_path):
    # a fresh interpreter pointed at a package copy without libmcx.so must
    # raise instead of computing anything another way
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1711_03244_amd"
    pkg.mkdir()
    src = os.path.join(ROOT, "paper_1711_03244_amd")
    for f in ["__init__.py", "mcx.py", "nn.py", "workloads.py"]:
        shutil.copy(os.path.join(src, f), pkg / f)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1711_03244_amd import mcx\n"
            "try:\n    mcx.lib()\nexcept RuntimeError as e:\n    print('RAISED', e)\n"
            % str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "RAISED" in r.stdout and "missing" in r.stdout, r.stdout + r.stderr

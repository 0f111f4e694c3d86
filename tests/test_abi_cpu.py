"""CPU checks of the C-ABI library: it loads, and exports every symbol include/*.h declares."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1711_07877_amd", "libsbd.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(sbd_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libsbd.so not built (run paper_1711_07877_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["sbd_plan", "sbd_apply", "sbd_free", "sbd_plan_info", "sbd_plan_export", "sbd_workspace_bytes",
              "sbd_plan_bytes", "sbd_strerror", "sbd_last_error", "sbd_default_options", "sbd_apply_parts",
              "sbd_fft2", "sbd_launch_times"]:
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_host_only_entry_points(lib):
    import paper_1711_07877_amd as pkg
    from paper_1711_07877_amd import _abi
    L = pkg.load_library()
    opt = _abi.sbd_options()
    L.sbd_default_options(ctypes.byref(opt))
    assert opt.max_rhs == 1 and opt.precision == 0 and opt.delta_min == 0.0
    assert L.sbd_strerror(-4).decode() == "tolerance below the SBD floor"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    ker = _abi.sbd_kernel(0, 0.0)
    st = L.sbd_plan(None, 10, ctypes.byref(ker), 1e-3, None, None, ctypes.byref(h))
    assert st == pkg._abi.SBD_EINVAL and not h.value
    st = L.sbd_plan(ctypes.c_void_p(16), 1, ctypes.byref(ker), 1e-3, None, None, ctypes.byref(h))
    assert st == pkg._abi.SBD_EINVAL
    assert L.sbd_workspace_bytes(None, 1) == 0
    L.sbd_free(None)


def test_struct_layouts_match_header(tmp_path):
    """Every field of the ctypes mirrors sits at the offset the C compiler gives it in
    include/sbd.h (a small host program compiled here prints sizeof and offsetof)."""
    from paper_1711_07877_amd import _abi
    import subprocess
    structs = {"sbd_kernel": _abi.sbd_kernel, "sbd_options": _abi.sbd_options, "sbd_info": _abi.sbd_info,
               "sbd_gmres_options": _abi.sbd_gmres_options}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sbd.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, str(src)], check=True)
    got = dict(ln.split() for ln in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_general_kernel_marshalling_and_checks():
    """SBD_GENERAL: the binding fills the kernel struct as include/sbd.h lays it out, and
    sbd_plan rejects a bad kernel description before any device call."""
    import paper_1711_07877_amd as pkg
    from paper_1711_07877_amd import _abi
    ker = pkg._kernel(pkg.SBD_GENERAL, 0.0, pkg.general_kernel(0.5, [(1, 7.0, 0.3, -0.2), (0, 2.0, 0.0, 1.0)], 3))
    assert (ker.kind, ker.c_log, ker.nterms, ker.enforce) == (2, 0.5, 2, 3)
    assert [ker.terms[i] for i in range(8)] == [1.0, 7.0, 0.3, -0.2, 0.0, 2.0, 0.0, 1.0]
    with pytest.raises(ValueError):
        pkg._kernel(pkg.SBD_GENERAL, 0.0, None)
    L = pkg.load_library()
    h = ctypes.c_void_p()
    bad = [pkg.general_kernel(1.0, [(0, 1.0, 1.0, 0.0)], 5), pkg.general_kernel(1.0, [(0.5, 1.0, 1.0, 0.0)], 1),
           pkg.general_kernel(1.0, [(9, 1.0, 1.0, 0.0)], 1), pkg.general_kernel(1.0, [(0, -1.0, 1.0, 0.0)], 1),
           pkg.general_kernel(float("nan"), [], 0), pkg.general_kernel(0.0, [], 0),
           pkg.general_kernel(1.0, [(0, 1.0, 1.0, 0.0)] * 9, 0)]
    for g in bad:
        k = pkg._kernel(pkg.SBD_GENERAL, 0.0, g)
        st = L.sbd_plan(ctypes.c_void_p(16), 10, ctypes.byref(k), 1e-3, None, None, ctypes.byref(h))
        assert st == _abi.SBD_EINVAL and not h.value
    assert "general kernel" in L.sbd_last_error().decode()


def test_host_tensors_are_refused_before_any_launch(lib):
    """A host tensor handed to the apply, the FFT or GMRES would give the kernels a host
    pointer (a GPU memory fault); the binding refuses it before calling the library."""
    import torch
    import paper_1711_07877_amd as pkg
    plan = pkg.Plan(None, 8, pkg.SBD_LAPLACE, 1)       # never reaches the library
    f = torch.zeros((1, 8), dtype=torch.float64)
    with pytest.raises(TypeError, match="CUDA"):
        plan.apply(f)
    with pytest.raises(TypeError, match="CUDA"):
        pkg.sbd_apply(plan, f, torch.zeros_like(f))
    with pytest.raises(TypeError, match="CUDA"):
        pkg.sbd_fft2(torch.zeros((4, 4), dtype=torch.complex64))
    with pytest.raises(TypeError, match="CUDA"):
        pkg.sbd_gmres(plan, torch.zeros(8, dtype=torch.float64))
    plan.handle = None

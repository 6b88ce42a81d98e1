"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes structures match the C layout, and host-only
entry points behave (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mag.h")


def _lib():
    from paper_2607_23354_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return L


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mag_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for required in ["mag_weighting", "mag_magnitude", "mag_create", "mag_destroy", "mag_dmin"]:
        assert required in names


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib()
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported by libmag.so"
        assert name in L.SIGNATURES, f"{name} has no ctypes signature"
    # nothing bound that the header does not declare
    assert set(L.SIGNATURES) <= set(declared_functions())


def test_enum_values_match_binding():
    L = _lib()
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    found = dict(re.findall(r"\b(MAG_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    for name in ["MAG_AUTO", "MAG_FP64_DENSE", "MAG_FP32_IR", "MAG_HODLR", "MAG_HSS", "MAG_FP64_CHOL"]:
        assert int(found[name]) == getattr(L, name), name


def test_struct_layouts_match_c(tmp_path):
    L = _lib()
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mag.h"\n'
        "int main(void){\n"
        'printf("%zu %zu\\n", sizeof(mag_opts), sizeof(mag_info));\n'
        'printf("%zu %zu %zu %zu %zu\\n", offsetof(mag_opts, tol), offsetof(mag_opts, seed),'
        " offsetof(mag_opts, inner_prec), offsetof(mag_info, argmin_w), offsetof(mag_info, n_update));\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(mag_eig_opts), sizeof(mag_eig_info), offsetof(mag_eig_opts, rtol),'
        " offsetof(mag_eig_info, iters_max), offsetof(mag_eig_info, solve_steps));\n"
        'printf("%zu %zu %zu\\n", sizeof(mag_tplus_opts), offsetof(mag_tplus_opts, method),'
        " offsetof(mag_tplus_opts, lo_factor));\n"
        'printf("%zu %zu %zu %zu %zu\\n", offsetof(mag_opts, diag), offsetof(mag_info, solver),'
        " offsetof(mag_info, backward_err), offsetof(mag_info, cond_est), offsetof(mag_opts, power_iters));\n"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    (so, si, o_tol, o_seed, o_ip, o_arg, o_nu, seo, sei, o_rt, o_im, o_ss, sto, o_me, o_lf,
     o_dg, o_sv, o_be, o_ce, o_pw) = map(int, out)
    assert o_dg == L.MagOpts.diag.offset and o_sv == L.MagInfo.solver.offset
    assert o_pw == L.MagOpts.power_iters.offset
    assert o_be == L.MagInfo.backward_err.offset and o_ce == L.MagInfo.cond_est.offset
    assert sto == ctypes.sizeof(L.MagTplusOpts) and o_me == L.MagTplusOpts.method.offset
    assert o_lf == L.MagTplusOpts.lo_factor.offset
    assert seo == ctypes.sizeof(L.MagEigOpts) and sei == ctypes.sizeof(L.MagEigInfo)
    assert o_rt == L.MagEigOpts.rtol.offset
    assert o_im == L.MagEigInfo.iters_max.offset and o_ss == L.MagEigInfo.solve_steps.offset
    assert so == ctypes.sizeof(L.MagOpts)
    assert si == ctypes.sizeof(L.MagInfo)
    assert o_tol == L.MagOpts.tol.offset
    assert o_seed == L.MagOpts.seed.offset
    assert o_ip == L.MagOpts.inner_prec.offset
    assert o_arg == L.MagInfo.argmin_w.offset
    assert o_nu == L.MagInfo.n_update.offset


def test_host_only_entry_points():
    L = _lib()
    lib = L.load()
    o = L.MagOpts()
    lib.mag_opts_default(ctypes.byref(o))
    assert o.tol == 1e-12 and o.gmres_restart == 30 and o.solver == L.MAG_AUTO
    assert o.inner_prec == 0  # every product with Z in FP64 unless asked
    assert lib.mag_padded_size(1) == 256
    assert lib.mag_padded_size(256) == 256
    assert lib.mag_padded_size(257) == 512
    assert lib.mag_padded_size(0) == 0
    for code in [0, -1, -2, -3, -4, -5, -6]:
        assert lib.mag_strerror(code)
    # NULL arguments are rejected before any device work
    assert lib.mag_create(None, 0) == L.MAG_EINVAL
    assert lib.mag_weighting(None, None, 10, 3, 1.0, None, None, None) == L.MAG_EINVAL
    assert lib.mag_dmin(None, None, 10, 3, None) == L.MAG_EINVAL
    assert lib.mag_set_stream(None, None) == L.MAG_EINVAL
    assert lib.mag_set_workspace_limit(None, 1 << 20) == L.MAG_EINVAL
    held = ctypes.c_uint64()
    assert lib.mag_workspace_bytes(None, ctypes.byref(held)) == L.MAG_EINVAL
    assert o.diag == 0  # no diagnostics unless asked
    assert o.power_iters == 0 and o.reserved_ == 0  # one Gaussian sample per level unless asked
    to = L.MagTplusOpts()
    lib.mag_tplus_opts_default(ctypes.byref(to))
    assert to.method == 0 and to.newton == 1  # bisection with safeguarded Newton unless asked
    eo = L.MagEigOpts()
    lib.mag_eig_opts_default(ctypes.byref(eo))
    assert eo.max_iter == 80 and eo.rtol == 1e-8
    ei = L.MagEigInfo()
    assert lib.mag_eig_extremes(None, None, 10, 3, 1.0, None, None, None, ctypes.byref(ei)) == L.MAG_EINVAL


def test_no_fallback_without_library(monkeypatch, tmp_path):
    from paper_2607_23354_amd import _lib as L
    saved = L._lib
    try:
        L._lib = None
        with pytest.raises(ImportError):
            L.load(str(tmp_path / "missing.so"))
    finally:
        L._lib = saved

"""The C-ABI library without a GPU: it builds, loads, exports every symbol that
include/wd.h declares, its struct layouts agree with the binding, and argument
errors are reported before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2111_14958_amd as wd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wd.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(wd.LIB_PATH):
        from paper_2111_14958_amd import build
        build.build()
    return wd.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(wd_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declarations_match_binding_list():
    assert declared_functions() == set(wd.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", wd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(wd_[a-z0-9_]+)\b", out))
    missing = declared_functions() - exported
    assert not missing, f"not exported: {sorted(missing)}"
    for name in declared_functions():
        assert hasattr(lib, name)


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "wd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(wd_cg_params), sizeof(wd_cg_report),
         sizeof(wd_tune_result), sizeof(wd_serve_config), sizeof(wd_request),
         sizeof(wd_serve_stats), offsetof(wd_request, params));
  return 0;
}
""")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(wd.CGParams), ctypes.sizeof(wd.CGReport), ctypes.sizeof(wd.TuneResult),
            ctypes.sizeof(wd.ServeConfig), ctypes.sizeof(wd.Request), ctypes.sizeof(wd.ServeStats),
            wd.Request.params.offset]
    assert got == want


def test_version_strerror_and_defaults(lib):
    assert lib.wd_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert lib.wd_strerror(code)
    p = wd.cg_default_params()
    assert p.tol == 1e-10 and p.max_iter == 20000 and p.reliable_every == 50
    assert p.inner == wd.F32 and p.use_x0 == 0 and p.persistent == -1


def test_argument_errors_need_no_device(lib):
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    h = ctypes.c_void_p()
    # bad time boundary sign, zero extent, null field: EINVAL before any device call
    assert lib.wd_gauge_create(dims, 0, ctypes.c_void_p(1), 0, None, ctypes.byref(h)) == wd.WD_EINVAL
    bad = (ctypes.c_int32 * 4)(4, 0, 4, 4)
    assert lib.wd_gauge_create(bad, -1, ctypes.c_void_p(1), 0, None, ctypes.byref(h)) == wd.WD_EINVAL
    assert lib.wd_gauge_create(dims, -1, None, 0, None, ctypes.byref(h)) == wd.WD_EINVAL
    assert b"t_sign" in lib.wd_last_error_detail() or lib.wd_last_error_detail() != b""
    assert lib.wd_dslash(None, 0.1, 0, None, None, 1, 0, None) == wd.WD_EINVAL
    assert lib.wd_cg_workspace_bytes(None, 1, None) == 0
    rep = wd.CGReport()
    assert lib.wd_cg_solve(None, 0.1, None, None, None, None, 0, ctypes.byref(rep), None) == wd.WD_EINVAL


def test_no_device_is_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    arch = ctypes.create_string_buffer(64)
    n = ctypes.c_int32()
    assert lib.wd_device_info(0, arch, 64, ctypes.byref(n)) == wd.WD_ENODEV


def test_no_oracle_in_product_path():
    """The HIP library and its binding never reference the oracle."""
    pkg = os.path.dirname(wd.__file__)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "wilson_oracle" not in text, f


def test_no_kernel_spills_to_scratch(lib):
    """The build records the compiler's per-kernel resource use and refuses
    kernels that spill registers to scratch memory."""
    from paper_2111_14958_amd import build
    if not os.path.exists(build.REPORT):
        build.build()
    lines = open(build.REPORT).read().splitlines()
    assert len(lines) > 50
    for line in lines:
        assert "scratch=0 " in line, line


def test_header_constants_match_binding():
    text = open(HEADER).read()
    defs = {m.group(1): m.group(2) for m in re.finditer(r"#define\s+(WD_[A-Z0-9_]+)\s+(.+?)\s*(?:/\*.*)?$",
                                                        text, flags=re.M)}
    want = {"WD_METHOD_CGNE": wd.METHOD_CGNE, "WD_METHOD_BICGSTAB": wd.METHOD_BICGSTAB,
            "WD_PRECOND_NONE": wd.PRECOND_NONE, "WD_PRECOND_EO": wd.PRECOND_EO,
            "WD_GAUGE_RECON12": wd.GAUGE_RECON12, "WD_FAMILY_CG_A": wd.FAMILY_CG_A,
            "WD_FAMILY_CG_B": wd.FAMILY_CG_B}
    for name, value in want.items():
        expr = defs[name].replace("u", "")
        assert eval(expr, {}) == value, (name, defs[name], value)

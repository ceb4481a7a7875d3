"""The C-ABI library loads and exports every symbol include/pstt2.h declares (CPU only).

No compute call is made here: this container has no GPU.  Host-side argument
validation that fails before touching the device is exercised too.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pstt2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:pstt2_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_and_binding_agree():
    from paper_2111_10448_amd import _lib as L
    assert _header_functions() == sorted(L.EXPORTS)


def test_library_exports_every_symbol():
    from paper_2111_10448_amd import _lib as L
    lib = L.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.pstt2_version()


def test_enums_match_header():
    """Every enumerator the header defines has the same value in the binding's tables."""
    from paper_2111_10448_amd import _lib as L
    src = open(os.path.join(ROOT, "include", "pstt2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {k: int(v) for k, v in re.findall(r"(PSTT2_\w+)\s*=\s*(-?\d+)", src)}
    for table, prefix in ((L.MID, "PSTT2_MID_"), (L.DRM, "PSTT2_DRM_"), (L.FN, "PSTT2_FN_"), (L.ALGO, "PSTT2_ALGO_")):
        names = {k[len(prefix):].lower(): v for k, v in vals.items() if k.startswith(prefix)}
        assert names == table, (prefix, names, table)
    assert vals["PSTT2_MID_TWOSIDED"] == 2


def test_struct_layouts_match_header(tmp_path):
    """Every field of the ctypes mirrors sits where gcc lays it out from the header."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    from paper_2111_10448_amd import _lib as L
    lines = []
    for ctype, cname in ((L.Desc, "pstt2_desc"), (L.TTCores, "tt_cores"), (L.Fn, "pstt2_fn")):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in ctype._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pstt2.h"\nint main(void) {\n' +
                   "\n".join(lines) + "\nreturn 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for ctype, cname in ((L.Desc, "pstt2_desc"), (L.TTCores, "tt_cores"), (L.Fn, "pstt2_fn")):
        assert int(got[cname]) == ctypes.sizeof(ctype), cname
        for fname, _ in ctype._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(ctype, fname).offset, (cname, fname)


def test_fn_layout_matches_the_c_compiler(tmp_path):
    """The same offsets as gcc lays out pstt2_fn from the header."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    from paper_2111_10448_amd import _lib as L
    src = tmp_path / "fn.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pstt2.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %d\\n", sizeof(pstt2_fn), offsetof(pstt2_fn, n_terms),'
                   ' offsetof(pstt2_fn, gamma), offsetof(pstt2_fn, centers), PSTT2_GAUSS_MAX_TERMS); return 0; }\n')
    exe = tmp_path / "fn"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(L.Fn), L.Fn.n_terms.offset, L.Fn.gamma.offset, L.Fn.centers.offset,
                   L.GAUSS_MAX_TERMS]


@pytest.mark.parametrize("field,value,msg", [
    ("d", 1, "d must be"),
    ("ell", 0, "ell must be"),
    ("ell", 33, "ell must be"),
    ("dtype", 7, "bad dtype"),
    ("mid", 3, "bad mid"),
])
def test_create_rejects_bad_descriptors(field, value, msg):
    from paper_2111_10448_amd import _lib as L
    lib = L.lib()
    d = L.Desc()
    d.d = 3
    for k in range(3):
        d.n[k] = 4
    d.ell = 4
    d.ranks[0] = 2
    d.ranks[1] = 2
    fac = np.zeros(64)
    d.drm_factors = fac.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    setattr(d, field, value)
    ctx = ctypes.c_void_p()
    st = lib.pstt2_create(ctypes.byref(d), None, ctypes.byref(ctx))
    assert st == L.EINVAL
    assert msg in lib.pstt2_last_error(None).decode()
    assert not ctx


def test_null_arguments_are_rejected():
    from paper_2111_10448_amd import _lib as L
    lib = L.lib()
    assert lib.pstt2_sketch(None, None, 0, 0) == L.EINVAL
    assert lib.pstt2_reset(None) == L.EINVAL
    out = ctypes.c_double()
    assert lib.tt_error(None, None, 0, ctypes.byref(out), None) == L.EINVAL
    lib.pstt2_destroy(None)
    lib.tt_cores_free(None)


def test_seeded_factor_query_validation():
    """pstt2_drm_factors (host only): the count, a short buffer and a bad order are reported."""
    from paper_2111_10448_amd import _lib as L
    lib = L.lib()
    d = L.Desc()
    d.d = 3
    d.n[0], d.n[1], d.n[2] = 4, 5, 6
    d.ell = 3
    cnt = ctypes.c_int64(0)
    assert lib.pstt2_drm_factors(ctypes.byref(d), None, ctypes.byref(cnt)) == L.OK
    assert cnt.value == (4 + 5 + 5 + 6) * 3          # psi_1, psi_2, omega_2, omega_3
    buf = (ctypes.c_double * 10)()
    cnt.value = 10
    assert lib.pstt2_drm_factors(ctypes.byref(d), buf, ctypes.byref(cnt)) == L.EINVAL
    assert "fewer" in lib.pstt2_last_error(None).decode()
    d.drm = L.DRM["independent"]
    assert lib.pstt2_drm_factors(ctypes.byref(d), None, ctypes.byref(cnt)) == L.OK
    assert cnt.value == ((4 + 5 + 6) + (4 + 5 + 6)) * 3   # split 1: psi_1, omega_2, omega_3; split 2: psi_1, psi_2, omega_3
    d.d = 1
    assert lib.pstt2_drm_factors(ctypes.byref(d), None, ctypes.byref(cnt)) == L.EINVAL

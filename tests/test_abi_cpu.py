"""CPU checks of the C-ABI library: it loads without a GPU, exports every
function include/svds.h declares, and the host-only entry points work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svds.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svds_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1607_01404_amd as P
    return P.load_library()


def test_header_declares_entry_points():
    names = _declared()
    for want in ("svds_opts_init", "svds_error_string", "svds_matrix_create", "svds_matrix_destroy",
                 "svds_matrix_spmm", "svds_solve", "svds_solve_prepared", "svds_small_eig",
                 "svds_small_svd"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_opts_defaults(lib):
    import paper_1607_01404_amd as P
    o = P.opts_init()
    assert o.max_basis_size == 0 and o.min_restart_size == 0 and o.block_size == 0
    assert o.max_prev_retain == -1 and o.two_sided_cleanup == 1 and o.precision == P.FP64
    assert lib.svds_opts_init(None) == -1


def test_error_strings():
    import paper_1607_01404_amd as P
    assert P.error_string(0) == "ok"
    assert "CSR" in P.error_string(-2)
    assert P.error_string(12345) == "unknown status"


def test_struct_layouts_match_header(tmp_path):
    import shutil
    import subprocess
    import paper_1607_01404_amd._lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "svds.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %d\\n",sizeof(svds_opts),'
                   'sizeof(svds_stats),sizeof(svds_csr),sizeof(svds_lpc_set),'
                   'offsetof(svds_opts,pc_model),SVDS_LPC_NPARAMS);return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert [int(x) for x in out] == [ctypes.sizeof(L.Opts), ctypes.sizeof(L.Stats),
                                     ctypes.sizeof(L.Csr), ctypes.sizeof(L.LpcSet),
                                     L.Opts.pc_model.offset, L.LPC_NPARAMS]


def test_null_arguments_rejected(lib):
    assert lib.svds_matrix_create(None, None, None) == -1
    assert lib.svds_solve_prepared(None, 1, 0, 1e-10, None, None, None, 1, None, 1, None, None, 0,
                                   None, None) == -1
    import ctypes as C
    nb = C.c_size_t(7)
    assert lib.svds_workspace_size(None, 1, 0, None, C.byref(nb)) == -1 and nb.value == 7
    assert lib.svds_workspace_size(None, 1, 0, None, None) == -1
    assert lib.svds_stream_release(None) == 0  # nothing kept for the default stream yet
    assert lib.svds_matrix_normal(None, 4, None, None, 1, None, None) == -1
    assert lib.svds_matrix_spmm(None, 0, 4, None, None, None) == -1


def test_every_field_offset_matches_header(tmp_path):
    """Each ctypes field of the option, statistics and CSR structs sits at the
    offset the C compiler gives it."""
    import shutil
    import subprocess
    import paper_1607_01404_amd._lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [("svds_opts", L.Opts), ("svds_stats", L.Stats), ("svds_csr", L.Csr),
               ("svds_lpc_set", L.LpcSet)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "svds.h"', 'int main(){']
    expect = []
    for cname, cls in structs:
        for fname, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(cls, fname).offset)
    lines.append("return 0;}")
    src = tmp_path / "off.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "off"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).decode().split()]
    assert got == expect

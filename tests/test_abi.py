"""The C-ABI library loads and exports every function include/*.h declares (CPU only)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2012_00357_amd", "libdd.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w ]*?[\s\*]+(dd_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_api():
    names = declared_functions()
    for must in ("dd_dataset_create", "dd_dataset_create_streamed", "dd_dataset_destroy",
                 "dd_project", "dd_project_noalloc", "dd_solve", "dd_server_create", "dd_server_submit", "dd_server_wait",
                 "dd_server_cancel", "dd_server_stats", "dd_server_destroy", "dd_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_binding_names_match_abi():
    from paper_2012_00357_amd import _lib
    for n in declared_functions():
        assert hasattr(_lib, n), f"binding lacks {n}"
    assert _lib.dd_version().startswith("libdd")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_has_no_oracle_dependency():
    """The product library links nothing from the oracle."""
    import subprocess
    out = subprocess.run(["ldd", LIB], capture_output=True, text=True).stdout
    assert "oracle" not in out


def test_struct_layouts_match_header():
    """The binding's ctypes structures have the sizes the C compiler gives the
    header's structures (a mismatch would corrupt every call)."""
    import subprocess
    import tempfile
    from paper_2012_00357_amd import _lib
    names = ["dd_dataset_opts", "dd_project_stats", "dd_project_opts", "dd_mesh", "dd_solve_opts",
             "dd_solve_result", "dd_server_opts", "dd_solve_request", "dd_server_statistics",
             "dd_index_info"]
    src = "#include <stdio.h>\n#include \"dd.h\"\nint main(void){\n" + "".join(
        f'printf("%zu\\n", sizeof({n}));\n' for n in names) + "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "sz.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "sz")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    for n, sz in zip(names, sizes):
        assert ctypes.sizeof(getattr(_lib, n)) == sz, n

"""Host-side checks of the C ABI (no GPU calls): the library loads and exports
every entry point that include/airga.h declares, and the binding wraps each."""
import os
import re
import subprocess

import pytest

from paper_1606_01216_amd import airga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "airga.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^AIRGA_API\s+[\w\s\*]*?\b(airga_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("airga_create", "airga_set_pencil", "airga_assemble_shift", "airga_spai_build",
                 "airga_spai_update", "airga_pcg_solve", "airga_prec_release"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(airga.LIB_PATH):
        pytest.skip("libairga.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", airga.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    # nothing but the C ABI is exported
    assert all(n.startswith("airga_") for n in exported), sorted(exported)


def test_binding_wraps_every_declared_symbol():
    assert sorted(airga.EXPORTED) == declared()


def test_library_loads_and_answers_host_only_calls():
    if not os.path.exists(airga.LIB_PATH):
        pytest.skip("libairga.so not built")
    h = airga.lib()
    assert h.airga_version().decode().count(".") == 2
    assert h.airga_kernel_count() > 0
    assert h.airga_kernel_name(0).decode() == "dir_spmv"
    o = airga.PcgOpts()
    h.airga_pcg_opts_default(o)
    assert o.tol == 1e-10 and o.mode == airga.MODE_FP64 and o.use_graph == 1
    s = airga.SpaiOpts()
    h.airga_spai_opts_default(s)
    assert s.tol == 0.01 and s.equilibrate == 1 and s.symmetrize == 1
    assert s.mr_iters == 0 and s.lfil == 0


def test_null_context_is_rejected_without_a_gpu():
    if not os.path.exists(airga.LIB_PATH):
        pytest.skip("libairga.so not built")
    h = airga.lib()
    info = airga.PencilInfo()
    st = h.airga_get_pencil_info(None, info)
    assert st == airga.EINVAL
    assert b"null context" in h.airga_last_error()

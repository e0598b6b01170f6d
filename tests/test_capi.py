"""C ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects invalid arguments on the host before any device work."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2404_16039_amd import lib
    decl = _declared()
    assert decl, "no declarations parsed"
    missing = [n for n in sorted(decl) if not hasattr(lib._lib, n)]
    assert not missing, missing
    # and the binding wraps every declared entry point under the same name
    assert decl <= set(lib.exported_symbols())
    assert lib.version() >= 10000


def test_host_validation_without_gpu():
    from paper_2404_16039_amd import lib
    L = lib._lib
    bad = lib.Pages(5, 5, 10, 1, 5, 25)
    rc = L.pf_page_det(lib.F32, C.byref(bad), C.c_void_p(16), C.c_void_p(16), None, None, None, None)
    assert rc == 3 and "1..4" in lib.last_error()
    nonsq = lib.Pages(2, 3, 10, 1, 2, 6)
    assert L.pf_page_det(lib.F32, C.byref(nonsq), C.c_void_p(16), C.c_void_p(16), None, None, None, None) == 3
    neg = lib.Pages(3, 3, -1, 1, 3, 9)
    assert L.pf_page_inv(lib.F64, C.byref(neg), C.c_void_p(16), C.byref(neg), C.c_void_p(16), None, None, None,
                         None, None) == 1
    ok = lib.Pages(3, 3, 10, 1, 3, 9)
    assert L.pf_page_det(7, C.byref(ok), C.c_void_p(16), C.c_void_p(16), None, None, None, None) == 2
    # empty batches are accepted without touching the device
    empty = lib.Pages(3, 3, 0, 1, 3, 9)
    assert L.pf_page_det(lib.F32, C.byref(empty), None, None, None, None, None, None) == 0
    assert L.pf_page_mtimes(lib.F64, C.byref(empty), None, 0, C.byref(empty), None, 0, C.byref(empty), None,
                            None) == 0
    # mismatched product shapes
    a = lib.Pages(3, 2, 4, 1, 3, 6)
    b = lib.Pages(3, 3, 4, 1, 3, 9)
    c = lib.Pages(3, 3, 4, 1, 3, 9)
    assert L.pf_page_mtimes(lib.F64, C.byref(a), C.c_void_p(16), 0, C.byref(b), C.c_void_p(16), 0, C.byref(c),
                            C.c_void_p(16), None) == 3
    # broadcast output is rejected
    cb = lib.Pages(3, 3, 4, 1, 3, 0)
    assert L.pf_page_transpose(lib.F64, C.byref(c), C.c_void_p(16), C.byref(cb), C.c_void_p(16), None) == 1
    # element calls: bad dimension, empty mesh
    assert L.pf_elem_geometry(4, lib.F32, 10, C.c_void_p(16), 5, C.c_void_p(16), None, None, None, None, None,
                              None, None, None, None) == 3
    assert L.pf_elem_stiffness_mass(3, lib.F32, 0, None, 0, None, None, None, None, None, None, None, None,
                                    None) == 0
    assert L.pf_boundary_normals(3, 9, 10, C.c_void_p(16), 2, C.c_void_p(16), None, None, None) == 2


def test_csr_handle_states_without_gpu():
    from paper_2404_16039_amd import lib
    L = lib._lib
    h = C.c_void_p()
    assert L.pf_csr_create(C.byref(h)) == 0 and h.value
    nn, nnz = C.c_int64(), C.c_int64()
    assert L.pf_csr_info(h, C.byref(nn), C.byref(nnz), None, None) == 9  # not built
    assert L.pf_assemble(h, lib.F32, None, None, None, None, None, None, None, None, None) == 9
    assert L.pf_csr_symbolic(h, 5, 1, 1, C.c_void_p(16), None) == 3
    assert L.pf_csr_symbolic(h, 3, -1, 1, C.c_void_p(16), None) == 1
    assert L.pf_csr_symbolic(h, 3, 1 << 31, 1, C.c_void_p(16), None) == 7
    # stage timing: null arguments, and timing off needs no device
    ns = len(lib.Csr.CSR_STAGES)
    ms = (C.c_double * ns)(*([1.0] * ns))
    calls = C.c_int64(-1)
    assert L.pf_csr_set_timing(None, 1) == 1
    assert L.pf_csr_stage_times(None, ms, None) == 1
    assert L.pf_csr_stage_times(h, None, None) == 1
    assert L.pf_csr_set_timing(h, 0) == 0
    assert L.pf_csr_stage_times(h, ms, C.byref(calls)) == 0 and calls.value == 0 and list(ms) == [0.0] * ns
    # load vector and energies: null / unbuilt handles and bad rules are host errors
    assert L.pf_rhs(None, lib.F32, None, None, 2, None, None, None, None, None, None) == 1
    assert L.pf_rhs(h, lib.F32, None, None, 2, None, None, None, None, None, None) == 9
    assert L.pf_energies(None, lib.F32, None, None, 2, None, None, None, None, None, None, None, None, None) == 1
    assert L.pf_energies(h, lib.F32, None, None, 2, None, None, None, None, None, None, None, None, None) == 9
    stages = re.search(r"#define PF_CSR_STAGES (\d+)", open(os.path.join(ROOT, "include", "pagefem.h")).read())
    assert int(stages.group(1)) == len(lib.Csr.CSR_STAGES) == 4
    L.pf_csr_destroy(h)
    L.pf_csr_destroy(None)


def test_plan_host_validation_without_gpu():
    from paper_2404_16039_amd import lib
    L = lib._lib
    h = C.c_void_p()
    assert L.pf_plan_create(7, 4, None, C.byref(h)) == 2
    assert L.pf_plan_create(lib.F32, 0, None, C.byref(h)) == 1
    assert L.pf_plan_create(lib.F32, 4, None, None) == 1
    assert L.pf_plan_set_groups(None, None, 0) == 1
    assert L.pf_plan_run(None, None, None) == 1
    assert L.pf_plan_launch(None, None, None) == 1
    assert L.pf_plan_tune(None, None, 0, None) == 1
    assert L.pf_plan_get_schedule(None, None) == 1
    assert L.pf_plan_info(None, None, None, None) == 1
    L.pf_plan_destroy(None)


def test_server_host_validation_without_gpu():
    from paper_2404_16039_amd import lib
    L = lib._lib
    h = C.c_void_p()
    assert L.pf_server_create(0, 4, 0, C.byref(h)) == 1
    assert L.pf_server_create(1 << 30, 0, 0, C.byref(h)) == 1
    assert L.pf_server_create(1 << 30, 4, 8, C.byref(h)) == 1
    assert L.pf_server_create(1 << 30, 4, 0, None) == 1
    assert L.pf_server_submit(None, None, None) == 1
    assert L.pf_server_poll(None, 1, None) == 1
    assert L.pf_server_drain(None) == 1
    assert L.pf_server_stats(None, None) == 1
    L.pf_server_destroy(None)


def test_server_footprint_without_gpu():
    from paper_2404_16039_amd import lib
    small = lib.server_footprint(3, lib.F32, 729, 3072)
    big = lib.server_footprint(3, lib.F32, 9261, 48000)
    assert 0 < small < big
    assert lib.server_footprint(2, lib.F64, 100, 162) > lib.server_footprint(2, lib.F32, 100, 162)
    import pytest
    with pytest.raises(lib.PagefemError):
        lib.server_footprint(5, lib.F32, 10, 10)

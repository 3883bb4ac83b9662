"""The C ABI without a GPU: the built library loads, exports every function that
include/lmbd.h declares, the binding declares the same set, and the calls that
need no device behave as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmbd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(lmbd_\w+)\s*\(", text))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_06409_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblmbd.so not built")
    return _lib.lib()


def test_header_declares_the_expected_api():
    names = header_functions()
    for must in ("lmbd_create", "lmbd_destroy", "lmbd_compute", "lmbd_compute_batch", "lmbd_estimate_footprint",
                 "lmbd_submit", "lmbd_poll", "lmbd_wait", "lmbd_server_create", "lmbd_server_destroy"):
        assert must in names


def test_library_exports_every_declared_function(lib):
    from paper_2407_06409_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s+(lmbd_\w+)$", out.stdout, flags=re.M))
    declared = header_functions()
    assert declared <= exported, declared - exported
    assert set(_lib.EXPORTED) == declared


def test_calls_that_need_no_device(lib):
    from paper_2407_06409_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "lmbd.h")).read()
    assert lib.lmbd_abi_version() == _lib.ABI_VERSION == int(re.search(r"LMBD_ABI_VERSION (\d+)", hdr).group(1))
    # the ctypes mirrors list the members of the header's structures in order
    for cname, mirror in (("lmbd_params", _lib.Params), ("lmbd_structure", _lib.StructureDesc),
                          ("lmbd_server_config", _lib.ServerConfig)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), hdr, flags=re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        members = [re.sub(r"\[.*\]", "", d.split()[-1]).lstrip("*") for d in body.split(";") if d.strip()]
        assert [f for f, _ in mirror._fields_] == members, cname
    assert lib.lmbd_status_string(0) == b"ok"
    assert lib.lmbd_status_string(8).startswith(b"a spectrum bound")
    assert lib.lmbd_status_string(3) == b"request exceeds the memory budget"
    assert lib.lmbd_status_string(7) == b"request cancelled"
    assert lib.lmbd_stage_name(3) == b"scs_assemble_factor_solve"
    assert lib.lmbd_stage_name(4) == b"scs_refine"
    assert lib.lmbd_stage_name(2) == b"scs_rhs"
    assert lib.lmbd_stage_name(10) is None
    assert lib.lmbd_last_error(None) == b""
    lib.lmbd_destroy(None)
    lib.lmbd_server_destroy(None)
    # NULL handles and out-pointers are argument errors, not crashes
    assert lib.lmbd_create(0, None) == 1
    assert lib.lmbd_compute_batch(None, None, 0, None, 0, None, 0, None) == 1
    assert lib.lmbd_set_memory_budget(None, 0) == 1
    assert lib.lmbd_set_mbd_product(None, 0) == 1
    assert lib.lmbd_submit(None, None, None) == 1
    assert lib.lmbd_poll(None, 0, None) == 1
    assert lib.lmbd_release(None, 0) == 1
    assert lib.lmbd_estimate_footprint(None, 0, None, None) == 1


def test_bad_device_index_is_an_argument_error(lib):
    h = ctypes.c_void_p()
    assert lib.lmbd_create(-1, ctypes.byref(h)) == 1
    assert lib.lmbd_create(1 << 20, ctypes.byref(h)) == 1


def test_radii_out_of_order_are_argument_errors(lib):
    """r_nbr >= r_mbd1 >= r_mbd2 (Sec. III.A) is checked before anything touches a device."""
    import numpy as np
    from paper_2407_06409_amd import api, LmbdError
    from workloads import frequency_grid
    g = frequency_grid(12)
    prm = api.MethodParams(omega=g[0], weight=g[1])
    base = dict(pos=np.array([[0.0, 0, 0], [2.0, 0, 0]]), species=np.array([1, 1], np.int32),
                v_ratio=np.array([0.9, 0.8]), cell=None, pbc=(0, 0, 0))
    for cut in (dict(r_scs=4.0, r_nbr=5.0, r_mbd1=4.0, r_mbd2=4.5),     # r_mbd1 < r_mbd2
                dict(r_scs=4.0, r_nbr=4.0, r_mbd1=5.0, r_mbd2=3.0)):    # r_nbr < r_mbd1
        with pytest.raises(LmbdError) as ei:
            api.estimate_footprint([dict(base, cutoffs=cut)], prm)
        assert ei.value.code == "LMBD_E_INVALID_ARG"

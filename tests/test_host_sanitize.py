"""The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a copy of the library built with both on its host code runs
tests/sanitize_driver.c, which checks arguments and strings and estimates the
footprint of open, periodic, slab, small self-image, two-radius, production-radii
and two-body-radii structures (host neighbour counting, form choice, workspace
layout), alone and as one batch.  Any sanitizer report fails the run.  The device
code is not exercised here: it runs in the GPU tests."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


def _structures():
    out = []
    st, cut = C.config_small_open()
    out.append((st, [cut["r_scs"], cut["r_nbr"], cut["r_mbd1"], cut["r_mbd2"], 0.0, 0.0]))
    st = C.carbon_box(216, 21)
    out.append((st, [4.0, 8.5, 5.0, 3.5, 0.0, 0.0]))                 # two radii, sparse form
    out.append((C.carbon_slab(36, 43, 8.0, 4.5, pbc=(1, 1, 0)), [4.0, 5.0, 5.0, 4.0, 0.0, 0.0]))
    out.append((C.hcno_box(50, 7050), [5.0, 5.0, 5.0, 5.0, 0.0, 0.0]))   # atoms see their own images
    out.append((C.carbon_box(128, 31), [4.0, 10.0, 6.0, 4.0, 10.0, 5.0]))  # K beyond LDS, two-body radii
    # production radii on a 12.9 A box: K of about 2,450 sites, most of them periodic images
    # (a batch above about 1,000 atoms needs the device for the sort's scratch size)
    out.append((C.carbon_box(216, 22), [4.0, 18.0, 10.0, 8.0, 0.0, 0.0]))
    return out


def _write(path):
    with open(path, "wb") as fh:
        items = _structures()
        fh.write(struct.pack("<i", len(items)))
        for st, radii in items:
            cell = np.zeros(9) if st.cell is None else np.asarray(st.cell, dtype=np.float64).ravel()
            pbc = [int(x) for x in st.pbc]
            fh.write(struct.pack("<i", st.n))
            fh.write(struct.pack("<3i", *pbc))
            fh.write(np.asarray(cell, "<f8").tobytes())
            fh.write(np.asarray(radii, "<f8").tobytes())
            fh.write(np.ascontiguousarray(st.pos, "<f8").tobytes())
            fh.write(np.ascontiguousarray(st.species, "<i4").tobytes())
            fh.write(np.ascontiguousarray(st.nu, "<f8").tobytes())


@pytest.mark.skipif(not (os.path.exists(CLANG) and shutil.which("/opt/rocm/bin/hipcc")), reason="needs the ROCm toolchain")
def test_host_code_under_address_and_undefined_behavior_sanitizers(tmp_path):
    from paper_2407_06409_amd.build import build_host_sanitized
    lib = build_host_sanitized(str(tmp_path))
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize_driver.c"),
                    lib, "-Wl,-rpath," + str(tmp_path), "-o", exe], check=True)
    data = str(tmp_path / "structures.bin")
    _write(data)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, data], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("ok")

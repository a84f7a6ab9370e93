"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU).

The library is rebuilt with -fsanitize=address,undefined on its host code
(device code as usual, no recovery from undefined behaviour) and the
host-only entry points are exercised through it in a child Python process
that preloads the sanitizer runtime: argument, mesh and geometry errors,
reference tables, numbering and patch lists (tests/test_library_host.py).
By default every host test but the reference-table parity runs, plus four
table cases (2D CG_4, 3D CG_4, Ned_3, RT_3); with RZ_HEAVY_TESTS=1 every
host test does.  Any sanitizer report fails the
child and so this test.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_entry_points_clean_under_asan_ubsan():
    if not shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) or not os.path.exists("/opt/rocm/llvm"):
        pytest.skip("hipcc or the ROCm clang runtime is missing")
    from paper_2506_17406_amd import build
    with tempfile.TemporaryDirectory(prefix="rz_hostsan_") as tmp:
        lib = build.build_host_sanitized(tmp)
        env = dict(os.environ)
        env.update(LD_PRELOAD=build.sanitizer_runtime(), RZ_LIBRARY=lib,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=97",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
        host = os.path.join("tests", "test_library_host.py")
        tables = ["2-CG-4", "3-CG-4", "3-Ned-3", "3-RT-3"]
        others = ["test_header_symbols_exported", "test_reference_argument_errors", "test_numbering_mesh_errors",
                  "test_setup_rejects_before_device_work", "test_numbering_bit_exact",
                  "test_vertex_star_lists_bit_exact", "test_comparator_lists_bit_exact",
                  "test_hdiv_curl_potential_entries", "test_hiptmair_decompositions_need_a_derivative_space",
                  "test_derivative_entries_left_out_of_the_hodge_csr"]
        sel = [host] if os.environ.get("RZ_HEAVY_TESTS") else (
            [host + "::test_reference_tables_match_oracle[%s]" % t for t in tables] +
            [host + "::" + f for f in others])
        proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider"] + sel,
                              cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
        out = proc.stdout + proc.stderr
        assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
        assert proc.returncode == 0, out[-4000:]
        assert " passed" in out, out[-2000:]
        print(out.strip().splitlines()[-1])

"""CPU checks of the library's host logic for the symbolic phase (no GPU): table capacities, the
owner tiles grown over contiguous row ranges, and the choice of the short-row kernel's hash
multiplier.  The functions live in paper_1905_08423_amd/csrc/host_logic.hpp, which the library
includes; tests/host_logic_check.cpp exercises them and is built here with g++."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_logic_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host_logic") / "host_logic_check")
    r = subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-Wall", "-Werror",
                        os.path.join(HERE, "host_logic_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_host_logic(host_logic_exe):
    r = subprocess.run([host_logic_exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    assert not any(l.startswith("FAIL") for l in lines), r.stdout
    for want in ["ok capacities", "ok tiles 27pt_40", "ok tiles 27pt_64 ", "ok tiles chain_100003",
                 "ok tiles random_long_rows", "ok hash multiplier 64^3", "ok hash multiplier 108^3",
                 "ok hash multiplier edge cases", "ok owner layout aligned", "ok fold estimate"]:
        assert any(l.startswith(want) for l in lines), (want, r.stdout)
    # the chain of 100,003 rows is split into three unequal ranges
    assert any("chain_100003 (100003 rows, 3 ranges" in l for l in lines), r.stdout

"""Grow's move table (make_moves in kernels.hpp, built at compile time) against
the brick geometry for n = 1..6: a host program (tests/move_table_check.cpp)
decodes every move from its index and checks, lane by lane, each quadrant's
membership, its target brick and the coded lane shift.  CPU only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_move_tables_match_brick_geometry(tmp_path):
    exe = str(tmp_path / "move_table_check")
    subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", "-w",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2508_13986_amd", "csrc"),
                    os.path.join(HERE, "move_table_check.cpp"), "-o", exe], check=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "move tables ok" in r.stdout

"""The C ABI used from a plain C program (host-only entry points; no GPU, no Python binding)."""
import os
import subprocess

import paper_1804_09764_amd as cc

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_c_program_against_the_abi(tmp_path):
    exe = str(tmp_path / "c_abi_host")
    libdir = os.path.dirname(cc.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "c_abi_host.c"), "-o", exe, "-L", libdir, "-lcc",
                           "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib", "-lm"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr

"""The C ABI used from plain C programs: host-only entry points (no GPU, no Python binding), and
the device entry points against closed forms on a GPU."""
import os
import subprocess

import pytest

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


@pytest.mark.gpu
def test_c_program_device_entry_points(tmp_path):
    """Graph preparation, colouring, plain and packed counts from plain C, against closed forms."""
    exe = str(tmp_path / "c_abi_device")
    libdir = os.path.dirname(cc.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                           os.path.join(HERE, "c_abi_device.c"), "-o", exe, "-L", libdir, "-lcc",
                           "-L", "/opt/rocm/lib", "-lamdhip64",
                           "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib", "-lm"])
    print("case: plain-C program over the device entry points", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr

"""The boundary as a plain C ABI: a C program that includes only
include/swvis.h is built with the system C compiler against libswvis.so and
run (host-side entry points; no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1909_03956_amd")


def test_c_program_uses_the_host_abi(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libswvis.so")):
        pytest.skip("libswvis.so not built")
    exe = tmp_path / "abi_host"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c", "abi_host.c"), "-o", str(exe),
                        "-L", PKG, "-lswvis", f"-Wl,-rpath,{PKG}", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all host checks passed" in r.stdout


@pytest.mark.gpu
def test_c_program_drives_the_device_abi(tmp_path):
    """Device entry points from C, with device memory from the HIP runtime's C
    API (the program prints each check before it runs the next)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cc = shutil.which("gcc") or shutil.which("cc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if cc is None or not os.path.exists(os.path.join(PKG, "libswvis.so")):
        pytest.skip("no C compiler or library")
    exe = tmp_path / "abi_device"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
                        os.path.join(ROOT, "tests", "c", "abi_device.c"), "-o", str(exe),
                        "-L", PKG, "-lswvis", f"-Wl,-rpath,{PKG}",
                        "-L", os.path.join(rocm, "lib"), "-lamdhip64",
                        f"-Wl,-rpath,{os.path.join(rocm, 'lib')}", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all device checks passed" in r.stdout

"""Host-side checks of the HIP library's index arithmetic (no GPU needed).

The shared-node enumeration and partial-slot layout of the assembly kernels
are compiled for the host from the same header the kernels include and checked
against a brute-force classification for many mesh / tile shapes."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_shared_node_enumeration(tmp_path):
    exe = str(tmp_path / "check_shared")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "--offload-arch=gfx950",
                           os.path.join(HERE, "host", "check_shared.hip"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert " 0 failures" in out.stdout

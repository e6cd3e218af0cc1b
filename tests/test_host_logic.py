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


def test_oracle_under_sanitizers(tmp_path):
    """The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc, CPU only) and driven through every entry point on small meshes of
    degree 1-4, several boundary patterns, both Heaviside laws and the mass
    shift; an invalid access, leak or undefined operation aborts the run."""
    exe = str(tmp_path / "oracle_sanitize")
    root = os.path.dirname(HERE)
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-D_GNU_SOURCE",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(root, "oracle", "oracle.c"),
                           os.path.join(HERE, "host", "oracle_sanitize.c"), "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(out.stdout[-2000:], out.stderr[-4000:])
    assert out.returncode == 0, out.stderr[-4000:]
    assert "0 failures" in out.stdout
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr

"""The C ABI from a C program (no Python or torch in its process): it builds
against include/raysh.h and links libraysh.so; without a GPU raysh_init
reports an error cleanly, with one its map equals the Python binding's,
pixel by pixel."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1703_09707_amd")
SRC = os.path.join(ROOT, "tests", "c_abi", "map_from_c.c")


def splitmix_stars(n, seed):
    """The star field map_from_c draws (splitmix64, as in the C source)."""
    mask = (1 << 64) - 1
    s = seed

    def nxt():
        nonlocal s
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    def unit():
        return (nxt() >> 11) * (1.0 / 9007199254740992.0)

    x, y, m = np.empty(n), np.empty(n), np.empty(n)
    for k in range(n):
        x[k] = 20.0 * unit() - 10.0
        y[k] = 20.0 * unit() - 10.0
        m[k] = 0.1 + 0.9 * unit()
    return x, y, m


@pytest.fixture(scope="module")
def program(tmp_path_factory):
    lib = os.path.join(PKG, "libraysh.so")
    if not os.path.exists(lib):
        pytest.fail("libraysh.so is not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    out = str(tmp_path_factory.mktemp("c_abi") / "map_from_c")
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", SRC, "-o", out, "-L", PKG, "-lraysh", f"-Wl,-rpath,{PKG}",
           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def test_c_program_builds_and_reports_errors_without_gpu(program):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([program, "100", "7"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, (r.stdout, r.stderr)
    assert r.stdout.startswith("raysh_init: code")


@pytest.mark.gpu
def test_c_program_map_equals_python_binding(program, tmp_path):
    import torch
    from paper_1703_09707_amd import raysh as R
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    map_file = str(tmp_path / "map.i32")
    r = subprocess.run([program, "300", "7", map_file], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
    _, binned, _, total, _, weighted = r.stdout.split()
    x, y, m = splitmix_stars(300, 7)
    rays = (-12.0, -12.0, 24.0 / 1024, 24.0 / 1024, 1024, 1024, 0, 0)
    pix = (-5.0, -5.0, 10.0 / 256, 10.0 / 256, 256, 256)
    with R.Context((0.1, 0.2, -0.05, x, y, m)) as ctx:
        counts, nb = ctx.map(rays, pix, "fp64", n_binned=True)
    from_c = np.fromfile(map_file, dtype=np.int32).reshape(256, 256)
    np.testing.assert_array_equal(from_c, counts.cpu().numpy())
    c = counts.cpu().numpy().astype(np.uint64).ravel()
    assert int(binned) == nb == int(c.sum()) == int(total)
    assert int(weighted) == int((c * np.arange(1, c.size + 1, dtype=np.uint64)).sum())

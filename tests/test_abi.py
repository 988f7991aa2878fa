"""The C ABI library loads and exports every entry point include/mlmc.h
declares (CPU only: no compute calls)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("mlmc_level", "mlmc_run", "mlmc_ctx_create", "mlmc_ctx_destroy", "mlmc_optimal_n"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1505_00965_amd import mlmc
    lib = mlmc.lib()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mlmc.EXPORTED) <= set(declared_symbols())


def test_library_exports_nothing_undeclared():
    import shutil
    import subprocess
    import pytest
    from paper_1505_00965_amd import mlmc
    if not shutil.which("nm"):
        pytest.skip("nm is not installed")
    out = subprocess.run(["nm", "-D", "--defined-only", mlmc.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines()
                if ln.split()[-1].startswith("mlmc_") and " T " in ln}
    assert exported == set(declared_symbols()), sorted(exported ^ set(declared_symbols()))


def test_null_context_is_rejected_without_a_gpu():
    from paper_1505_00965_amd import mlmc
    lib = mlmc.lib()
    assert lib.mlmc_set_launch(None, 0, 0) == mlmc.MLMC_EINVAL
    assert lib.mlmc_ctx_destroy(None) == mlmc.MLMC_OK
    assert lib.mlmc_last_error(None) == b"null context"


def test_oracle_and_library_share_no_source():
    # the oracle and the HIP path are independent: no includes either way
    import glob
    for f in glob.glob(os.path.join(ROOT, "paper_1505_00965_amd", "**", "*"), recursive=True):
        if f.endswith((".hip", ".hpp", ".cpp", ".h", ".py")):
            txt = open(f).read()
            assert "oracle" not in re.sub(r"#.*|//.*", "", txt).lower() or f.endswith("workloads.py"), f
    for f in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if f.endswith((".c", ".h", ".py")):
            assert "paper_1505_00965_amd" not in open(f).read(), f


def test_one_hip_runtime_per_process():
    """torch carries its own HIP runtime: the library must bind to that copy
    (two runtimes in one process leave torch without the device)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1505_00965_amd import mlmc\n"
            "mlmc.lib()\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "paths = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "print(len(paths))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"

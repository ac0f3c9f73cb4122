"""The C-ABI library loads without a GPU and exports every function that
include/sd.h declares (no device calls here)."""
import os
import re
import subprocess

from paper_2206_11664_amd import sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sd_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declarations_match_binding_list():
    assert declared_functions() == set(sd.EXPORTED)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", sd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = declared_functions() - exported
    assert not missing, missing
    L = sd.lib()
    for name in declared_functions():
        assert hasattr(L, name)


def test_status_strings_and_version():
    L = sd.lib()
    for s in range(8):
        assert L.sd_status_string(s).decode().startswith("SD_")
    assert "gfx950" in sd.sd_version()


def test_evolve_rejects_bad_arguments_without_device():
    # argument validation happens before any device work
    h = sd.sd_hamiltonian_create(2, ["XX", "ZZ"], [1.0, 0.5])
    p = sd.sd_plan(h)
    L = sd.lib()
    assert L.sd_evolve(p, None, 1, 0.1, 1, 1, None) == sd.SD_ERR_ARG
    assert L.sd_evolve(p, 8, 1, 0.1, 1, 3, None) == sd.SD_ERR_ARG          # order 3
    assert L.sd_evolve(p, 8, 1, 0.1, -1, 1, None) == sd.SD_ERR_ARG         # steps < 0
    assert L.sd_evolve(p, 8, 1, float("inf"), 1, 1, None) == sd.SD_ERR_ARG
    assert L.sd_evolve(p, 8, 7, 0.1, 1, 1, None) == sd.SD_ERR_ARG          # dtype
    assert L.sd_evolve(p, 8, 1, 0.1, 1, 1, None) == sd.SD_ERR_WORKSPACE    # nothing bound
    assert L.sd_bind_workspace(p, 8, 16, None) == sd.SD_ERR_WORKSPACE      # too small
    sd.sd_plan_destroy(p)
    sd.sd_hamiltonian_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    # the benchmark runs on one GPU; asking for more exits at once with a message
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

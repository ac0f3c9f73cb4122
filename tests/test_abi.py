"""The C-ABI library loads without a GPU and exports every function that
include/sd.h declares (no device calls here)."""
import ctypes
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


def test_library_never_allocates_device_memory():
    # the caller owns every device buffer: the library imports no HIP
    # allocation routine at all
    out = subprocess.run(["nm", "-D", "--undefined-only", sd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    imported = {l.split()[-1].split("@")[0] for l in out.splitlines() if l.strip()}
    for name in ("hipMalloc", "hipMallocAsync", "hipMallocManaged", "hipExtMallocWithFlags",
                 "hipMallocFromPoolAsync", "hipFree", "hipFreeAsync", "hipHostMalloc"):
        assert name not in imported, name


def test_reductions_and_autotune_validate_caller_memory_without_device():
    L = sd.lib()
    need = L.sd_reduction_scratch_bytes()
    assert need >= 8 * (2 * 2048 + 2)
    out = (ctypes.c_double * 2)()
    # null scratch, too small scratch, misaligned scratch: rejected before any device work
    assert L.sd_norm2(8, 0, 10, out, None, need, None) == sd.SD_ERR_ARG
    assert L.sd_norm2(8, 0, 10, out, 256, need - 8, None) == sd.SD_ERR_WORKSPACE
    assert L.sd_norm2(8, 0, 10, out, 260, need, None) == sd.SD_ERR_WORKSPACE
    assert L.sd_inner(8, 16, 1, 10, out, None, need, None) == sd.SD_ERR_ARG
    assert L.sd_inner(8, 16, 1, 10, out, 256, 16, None) == sd.SD_ERR_WORKSPACE
    assert L.sd_norm2(8, 0, 41, out, 256, need, None) == sd.SD_ERR_RANGE
    assert L.sd_inner(8, 16, 5, 10, out, 256, need, None) == sd.SD_ERR_ARG   # dtype
    # the variant with the library's static scratch: the same argument checks
    assert L.sd_inner_noalloc(None, 16, 1, 10, out, None) == sd.SD_ERR_ARG
    assert L.sd_inner_noalloc(8, 16, 1, 10, None, None) == sd.SD_ERR_ARG
    assert L.sd_inner_noalloc(8, 16, 1, 41, out, None) == sd.SD_ERR_RANGE
    assert L.sd_inner_noalloc(8, 16, 1, -1, out, None) == sd.SD_ERR_RANGE
    assert L.sd_inner_noalloc(8, 16, 5, 10, out, None) == sd.SD_ERR_ARG   # dtype
    # the autotuner's workspace: the largest plan workspace among the candidates
    h = sd.sd_hamiltonian_create(6, ["XXIIII", "ZZIIII", "IXXIII", "IIIZZZ"], [1.0, 0.5, 0.2, 0.3])
    ws = sd.sd_autotune_workspace_bytes(h, sd.SD_C64, [6, 7, 8])
    sizes = []
    for d in (6, 7, 8):
        o = sd.sd_plan_options_default()
        o.tile_log2_c64 = d
        o.coalesce_log2_c64 = min(4, d - 1)
        p = sd.sd_plan(h, o)
        sizes.append(sd.sd_plan_info_get(p).workspace_bytes)
        sd.sd_plan_destroy(p)
    assert ws == max(sizes)
    cand = (ctypes.c_int32 * 2)(6, 14)
    b = ctypes.c_int64()
    assert L.sd_autotune_workspace_bytes(h, None, 0, cand, 2, ctypes.byref(b)) == sd.SD_ERR_RANGE
    best = sd.sd_plan_options()
    cand = (ctypes.c_int32 * 1)(8)
    # no workspace: rejected before planning or device work
    assert L.sd_autotune_tiles(h, None, 0, 8, 0.1, 1, 1, cand, 1, None, 0, ctypes.byref(best), None,
                               None) == sd.SD_ERR_ARG
    sd.sd_hamiltonian_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    # the benchmark runs on one GPU; asking for more exits at once with a message
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

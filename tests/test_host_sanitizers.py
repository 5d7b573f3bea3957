"""The host side of the C ABI under the address and undefined-behaviour
sanitizers (no GPU needed): every library source is compiled with the
sanitizers on its host code only (`-Xarch_host`), linked with the checks in
tests/host_abi_check.c, and run. The checks walk configuration validation
and workspace planning over valid and invalid configurations (sphere
support and link capacity bounds, pipe-wall markers and links, size
limits) and the argument checks of the entry points with null handles and
pointers; the run must end cleanly, report nothing, and return the
expected statuses."""
import concurrent.futures as cf
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_1906_05448_amd" / "csrc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-fno-omit-frame-pointer"]

EXPECT = {
    "default": 0, "dense512_f16": 0, "dense1024_f32": 0, "too_many_nodes": -3, "f32_offset_limit": -3,
    "too_small": -1, "tau_half": -1, "rate_two": -1, "force_inf": -1, "bad_store": -1, "bad_bc": -1,
    "bad_lattice": -1, "ibb_128_98": 0, "ibb_linear": 0, "ibb_order3": -1, "ibm_128_98": 0, "ibm_rd0": 0,
    "ibm_rd_large": -1, "ibm_box_too_wide": -1, "ibm_iters": -1, "ibb_512_6250": 0, "ibm_512_6250": 0,
    "radius_box": -1, "particles_no_bc": -1, "restitution": -1, "pipe_ibb": 0, "pipe_d3q27": 0,
    "pipe_d3q27_bulk": 0, "pipe_d3q27_bad_bulk": -1, "pipe_d3q27_f16": -1, "pipe_ibm": 0,
    "pipe_radius_small": -1, "pipe_no_bc": -1, "d3q19_bulk": -1,
}


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not available")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, " ".join(cmd) + "\n" + res.stderr[-4000:]


def test_host_abi_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    inc = ["-I", str(ROOT / "include"), "-I", str(CSRC)]
    objs = []
    jobs = []
    for src in sorted(CSRC.glob("*.hip")):
        obj = tmp_path / (src.stem + ".o")
        objs.append(str(obj))
        jobs.append([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-c",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN, *inc, str(src), "-o", str(obj)])
    drv = tmp_path / "host_abi_check.o"
    jobs.append([hipcc, "-x", "c++", "-O1", "-g", "-c", *SAN, *inc, str(ROOT / "tests" / "host_abi_check.c"),
                 "-o", str(drv)])
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(_run, jobs))
    exe = tmp_path / "host_abi_check"
    _run([hipcc, "--offload-arch=gfx950", *SAN[:4], *objs, str(drv), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    got, texts = {}, []
    for ln in res.stdout.splitlines():
        parts = ln.split()
        if parts[0] == "strerror":
            texts.append(parts[2])
        else:
            got[parts[0]] = parts[1:]
    for name, st in EXPECT.items():
        assert int(got[name][0]) == st, (name, got[name])
        if st == 0:
            assert int(got[name][1]) > 0, name
    for name, v in got.items():
        if name.endswith("_null") or name.endswith("_n0"):
            assert int(v[0]) == -1, (name, v)
    assert texts and all(t == "text" for t in texts)

"""The C-ABI library loads and exports every symbol include/lbm.h declares;
host-only entry points (no GPU work) behave as documented."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "lbm.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = declared_functions()
    for core in ["lbm_init", "lbm_step", "lbm_destroy", "lbm_strerror", "lbm_workspace_size"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1906_05448_amd import lbm
    L = lbm.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_defaults_and_workspace_size():
    from paper_1906_05448_amd import lbm
    L = lbm.lib()
    c = lbm._CConfig()
    L.lbm_config_default(ctypes.byref(c))
    assert (c.nx, c.ny, c.nz) == (32, 32, 32)
    assert c.tau == 0.6 and c.s_e == 1.19 and c.s_m == 1.98 and c.ibm_iters == 2
    cfg = lbm.Config(nx=32, ny=32, nz=32)
    n = lbm.workspace_size(cfg)
    assert n >= 2 * 19 * 32 ** 3 * 4
    n16 = lbm.workspace_size(lbm.Config(nx=32, ny=32, nz=32, store=lbm.STORE_F16S))
    assert n16 < n


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau=0.4), dict(nx=3), dict(s_e=2.0), dict(s_m=0.0),
                                 dict(store=7)])
def test_invalid_config_rejected(bad):
    from paper_1906_05448_amd import lbm
    cfg = lbm.Config(**bad)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.workspace_size(cfg)
    assert ei.value.status == -1


def test_strerror_texts():
    from paper_1906_05448_amd import lbm
    L = lbm.lib()
    for s in range(-6, 1):
        assert L.lbm_strerror(s)
    assert L.lbm_strerror(-5).decode().startswith("numerical instability")

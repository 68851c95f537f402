"""The C-ABI library loads and exports every function include/lbm.h declares;
host-side argument validation (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1909_12390_amd import lbm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:lbm_status|void|const char\*)\s+(lbm_\w+)\s*\(", txt, re.M)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(lbm.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _mix():
    return {"a": [2 / 49, 0.08], "b": [2 / 21, 0.15], "omega": [0.1, 0.2], "M": [1.0, 1.6],
            "k": [[0, 0.01], [0.01, 0]], "R": 1.0}


def _bytes(**kw):
    args = dict(lattice="D2Q9", shape=(16, 20), T=0.05, tau=0.8, beta=1.5, gamma=[0.5, 1.0])
    args.update(kw)
    m = lbm.mixture_struct(args.pop("mix", _mix()))
    p = lbm.params_struct(**args)
    out = ctypes.c_size_t(0)
    code = lbm.lib().lbm_workspace_bytes(ctypes.byref(m), ctypes.byref(p), ctypes.byref(out))
    return code, out.value


def test_workspace_bytes_layout():
    code, n = _bytes()
    assert code == lbm.LBM_OK
    cells = 16 * 20
    assert n >= 2 * 2 * 9 * cells * 8 + cells * 8        # two float64 population copies + psi
    code16, n16 = _bytes(storage="f16")
    assert code16 == lbm.LBM_OK and n16 < n


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(G=0.0), dict(G=1.0), dict(gamma=[0.0, 1.0]), dict(gamma=[1.2, 1.0]),
    dict(shape=(0, 5)), dict(lattice="D3Q19", shape=(4, 4, 0)),
])
def test_host_validation_rejects(bad):
    code, _ = _bytes(**bad)
    assert code == lbm.LBM_ERR_ARG
    assert len(lbm.lib().lbm_last_error()) > 0


def test_host_validation_rejects_asymmetric_k_and_bad_nc():
    m = _mix()
    m["k"] = [[0, 0.01], [0.02, 0]]
    assert _bytes(mix=m)[0] == lbm.LBM_ERR_ARG
    m5 = {k: (v * 3 if isinstance(v, list) else v) for k, v in _mix().items()}
    m5["a"] = [0.04] * 5
    with pytest.raises(IndexError):
        lbm.mixture_struct(m5)      # more than LBM_MAX_NC components cannot be marshalled


def test_mrt_rates_checked():
    assert _bytes(collision="mrt", mrt_s=[1.0] * 9)[0] == lbm.LBM_OK
    assert _bytes(collision="mrt", mrt_s=[1.0] * 8 + [2.5])[0] == lbm.LBM_ERR_ARG

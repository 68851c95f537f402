"""The C-ABI library loads and exports every function include/lbm.h declares;
host-side argument validation (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
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


def _mix4():
    return {"a": [2 / 49, 0.08, 0.05, 0.06], "b": [2 / 21, 0.15, 0.1, 0.12], "omega": [0.1, 0.2, 0.15, 0.25],
            "M": [1.0, 1.6, 1.1, 1.3], "k": np.zeros((4, 4)).tolist(), "R": 1.0}


def _batch_layout(nboxes=2, tile=0, grid=0, graph_steps=0, nc=2, lattice="D2Q9", shape=(8, 16), gamma=None,
                  solid=None, psi_wall=0.0, storage=2, fused=0):
    n = nboxes
    arr = (lbm.LbmBox * max(n, 1))()
    for i in range(n):
        m = _mix() if nc == 2 else _mix4()
        arr[i].mix = lbm.mixture_struct(m)
        arr[i].nx, arr[i].ny, arr[i].nz = shape[1], shape[0], 1
        arr[i].T, arr[i].tau, arr[i].G, arr[i].beta = 0.06, 0.8, -1.0, 1.16
        for k, g in enumerate(gamma if gamma is not None else [0.5] * (nc - 1) + [1.0]):
            arr[i].gamma[k] = g
        if solid is not None and i == 0:
            arr[i].solid = solid.ctypes.data
            arr[i].psi_wall = psi_wall
    prm = lbm.LbmBatchParams()
    prm.lattice = lbm.LATTICES[lattice]
    prm.collision, prm.forcing, prm.storage = 0, 1, storage
    prm.tile, prm.grid, prm.graph_steps = tile, grid, graph_steps
    prm.fused = fused
    ws, fe, pe = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
    code = lbm.lib().lbm_batch_layout(arr, n, ctypes.byref(prm), ctypes.byref(ws), ctypes.byref(fe),
                                      ctypes.byref(pe))
    return code, ws.value, fe.value, pe.value


def test_fused_batch_validation():
    with open(HEADER) as fh:
        nx_max = int(re.search(r"#define LBM_FUSED_MAX_NX (\d+)", fh.read()).group(1))
    f64, f32, f16 = (lbm.STORAGES[k] for k in ("f64", "f32", "f16"))
    assert _batch_layout(fused=1, storage=f16)[0] == lbm.LBM_OK
    assert _batch_layout(fused=1, storage=f32)[0] == lbm.LBM_OK
    assert _batch_layout(fused=1, storage=f64)[0] == lbm.LBM_ERR_ARG
    assert _batch_layout(fused=1, lattice="D3Q19")[0] == lbm.LBM_ERR_ARG
    assert _batch_layout(fused=2)[0] == lbm.LBM_ERR_ARG
    assert _batch_layout(fused=1, shape=(2, nx_max))[0] == lbm.LBM_OK
    assert _batch_layout(fused=1, shape=(2, nx_max + 1))[0] == lbm.LBM_ERR_ARG
    assert _batch_layout(fused=0, shape=(2, nx_max + 1))[0] == lbm.LBM_OK


def test_batch_layout_counts_and_validation():
    code, ws, fe, pe = _batch_layout(nboxes=3)
    assert code == lbm.LBM_OK
    assert fe == 3 * 2 * 8 * 16 and pe == 9 * fe
    assert ws >= pe * 2 * 2 + fe * 4 * 2          # two f16 offset copies + float32 bases
    for bad in (dict(tile=512), dict(tile=100), dict(grid=-1), dict(graph_steps=-2), dict(nboxes=0),
                dict(gamma=[0.0, 1.0]), dict(gamma=[1.5, 1.0]), dict(lattice="D2Q9", shape=(0, 16))):
        assert _batch_layout(**bad)[0] == lbm.LBM_ERR_ARG, bad
        assert len(lbm.lib().lbm_last_error()) > 0


def test_eos_param_grad_validates():
    m = lbm.mixture_struct(_mix())
    z = np.zeros(4)
    out = np.zeros(4)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    assert lbm.lib().lbm_eos_param_grad(ctypes.byref(m), -1.0, dp(z), dp(z), dp(out), dp(out), dp(out)) \
        == lbm.LBM_ERR_ARG
    assert lbm.lib().lbm_eos_param_grad(ctypes.byref(m), 0.05, None, dp(z), dp(out), dp(out), dp(out)) \
        == lbm.LBM_ERR_ARG


def test_host_validation_rejects_planes_past_4gib():
    """One component's direction planes are addressed with 32-bit byte offsets:
    a box whose float64 planes would pass 4 GiB is refused on the host."""
    assert _bytes(lattice="D3Q19", shape=(310, 310, 310))[0] == lbm.LBM_ERR_ARG   # 19 x 8 x 2.98e7 B > 4 GiB
    assert _bytes(lattice="D3Q19", shape=(300, 300, 300))[0] == lbm.LBM_OK        # 19 x 8 x 2.70e7 B < 4 GiB
    assert _bytes(lattice="D3Q19", shape=(128, 128, 128))[0] == lbm.LBM_OK


def test_batch_walls_layout_and_validation():
    """Wall masks take 4 bytes per cell of the boxes that have walls, in the caller's
    workspace; a non-finite or negative wall psi is refused on the host."""
    solid = np.zeros((8, 16), dtype=np.uint8)
    solid[0] = 1
    code0, ws0, _, _ = _batch_layout(nboxes=3)
    code1, ws1, _, _ = _batch_layout(nboxes=3, solid=solid, psi_wall=0.5)
    assert code0 == lbm.LBM_OK and code1 == lbm.LBM_OK
    assert ws1 >= ws0 + 8 * 16 * 4
    for pw in (float("nan"), -0.1, float("inf")):
        assert _batch_layout(nboxes=2, solid=solid, psi_wall=pw)[0] == lbm.LBM_ERR_ARG


def test_context_calls_reject_null_handles():
    """Host-side argument checks of the calls added for walls, gamma updates and
    graph replay (no device needed)."""
    L = lbm.lib()
    g = np.full(4, 0.5)
    assert L.lbm_set_solid(None, None, ctypes.c_double(0.0)) == lbm.LBM_ERR_ARG
    assert L.lbm_set_graph_steps(None, 4) == lbm.LBM_ERR_ARG
    assert L.lbm_set_gamma(None, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lbm.LBM_ERR_ARG
    assert L.lbm_step(None, 1) == lbm.LBM_ERR_ARG


def test_batch_binding_checks_initial_field_shapes():
    """A box whose rho0 does not have (nc_b, *shape) is refused by the binding before
    anything reaches the library or the device."""
    mix = _mix()
    nc = len(mix["a"])
    good = {"mix": mix, "shape": (8, 16), "T": 0.07, "tau": 0.8, "beta": 1.3, "gamma": [0.5] * nc,
            "rho0": np.ones((nc, 8, 16))}
    bad = dict(good, rho0=np.ones((nc, 16, 8)))
    with pytest.raises(ValueError, match="box 1: rho0"):
        lbm.LbmBatch([good, bad], "D2Q9", storage="f16")


def test_batch_box_planes_past_4gib_refused():
    """A box's planes are addressed with 32-bit byte offsets: float64 one component's
    planes, the offset formats all components' interleaved planes. A box whose
    float64 planes fit but whose four-component float32 offsets would not is
    refused for float32 storage only."""
    shape = (6000, 6000)            # 9 x 8 x 3.6e7 B = 2.6 GB; x 4 components x 4 B = 5.2 GB
    assert _batch_layout(nboxes=1, nc=4, shape=shape, storage=lbm.STORAGES["f64"])[0] == lbm.LBM_OK
    assert _batch_layout(nboxes=1, nc=4, shape=shape, storage=lbm.STORAGES["f16"])[0] == lbm.LBM_OK
    assert _batch_layout(nboxes=1, nc=4, shape=shape, storage=lbm.STORAGES["f32"])[0] == lbm.LBM_ERR_ARG


def test_python_structs_match_the_c_header(tmp_path):
    """Every ctypes mirror of an lbm.h struct has the C struct's size and field
    offsets (compiled with the host C compiler against the header)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"lbm_mixture": lbm.LbmMixture, "lbm_params": lbm.LbmParams, "lbm_flash_result": lbm.LbmFlashResult,
             "lbm_box": lbm.LbmBox, "lbm_batch_params": lbm.LbmBatchParams}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbm.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)

"""Host logic of bench.py: algorithmic bytes, the stored-counter lookup keyed by the
step kernels' sources, the bulk-phase reading and the iso-fugacity residual, and
the refusal of more than one GPU."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes():
    # 2 nc Q s populations + 16 psi + 8 nc float32 base (offset formats only)
    assert bench.b_alg(4, 19, "f16") == 352
    assert bench.b_alg(4, 19, "f32") == 656
    assert bench.b_alg(4, 19, "f64") == 1232
    assert bench.b_alg(2, 9, "f64") == 304
    assert bench.b_alg(3, 9, "f32") == 2 * 3 * 9 * 4 + 16 + 24
    for st in ("f16", "f32", "f64"):
        assert bench.b_alg_collide(4, 19, st) == bench.b_alg(4, 19, st) - 8


def _copy_tree(tmp_path):
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_1909_12390_amd", "csrc"), root / "paper_1909_12390_amd" / "csrc")
    (root / "profiles").mkdir()
    return root


def test_counters_follow_the_step_kernel_sources(tmp_path, monkeypatch):
    root = _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(root / "profiles" / "traffic.json"))
    sha = bench.kernel_source_sha()
    assert sha == bench.kernel_source_sha() and len(sha) == 16
    rec = {"k": {"source_sha": sha, "bytes_per_launch": 1.0}}
    (root / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_profile("k") == rec["k"]
    assert bench.measured_profile("other") == {}
    # host-only sources do not void the record ...
    with open(root / "paper_1909_12390_amd" / "csrc" / "thermo.cpp", "a") as fh:
        fh.write("\n// host-only change\n")
    assert bench.kernel_source_sha() == sha and bench.measured_profile("k") == rec["k"]
    # ... a step kernel's source does
    with open(root / "paper_1909_12390_amd" / "csrc" / "lbm_kernels.hpp", "a") as fh:
        fh.write("\n// kernel change\n")
    assert bench.kernel_source_sha() != sha
    assert bench.measured_profile("k") == {}


def test_bulk_phases_of_a_drop():
    torch = pytest.importorskip("torch")
    shape = (16, 16, 16)
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    r = np.sqrt((x - 8.0) ** 2 + (y - 8.0) ** 2 + (z - 8.0) ** 2)
    M = np.array([1.0, 2.0])
    liq, vap = np.array([4.0, 2.0]), np.array([0.3, 0.1])          # cell-volume densities
    rho = np.where(r <= 4.0, 1.0, 0.0)[None] * liq[:, None, None, None] + \
        np.where(r <= 4.0, 0.0, 1.0)[None] * vap[:, None, None, None]
    out = bench.phase_mole_fractions(torch.as_tensor(rho), M, {"R0": 4.0}, shape)
    nl, nv = liq / M, vap / M
    assert np.allclose(out["liquid"], nl / nl.sum(), rtol=1e-14)
    assert np.allclose(out["vapor"], nv / nv.sum(), rtol=1e-14)
    assert np.allclose(out["n_liquid"], nl, rtol=1e-14) and np.allclose(out["n_vapor"], nv, rtol=1e-14)


def test_iso_fugacity_residual_of_the_flash_is_zero():
    from paper_1909_12390_amd import lbm
    mix = {"a": [2 / 49, 0.08], "b": [2 / 21, 0.15], "omega": [0.1, 0.2], "M": [1.0, 1.6],
           "k": [[0, 0.01], [0.01, 0]], "R": 1.0}
    Tc = lbm.lbm_critical(mix)[0]
    T = 0.8 * float(np.min(Tc))
    z = [0.5, 0.5]
    pb, pd = lbm.lbm_bubble_pressure(mix, T, z), lbm.lbm_dew_pressure(mix, T, z)
    fl = lbm.lbm_flash(mix, T, 0.5 * (pb + pd), z)
    n_l, n_v = fl.rho_l * np.asarray(fl.x[:2]), fl.rho_v * np.asarray(fl.y[:2])
    f_l, f_v, res, p = bench.fugacities(lbm, mix, T, n_l, n_v)
    assert res < 1e-20
    assert p == pytest.approx(0.5 * (pb + pd), rel=1e-10)
    f_l2, f_v2, res2, _ = bench.fugacities(lbm, mix, T, n_l, 1.05 * n_v)
    assert res2 > 1e-6                                   # a perturbed vapour is not in equilibrium


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_stored_counters_match_the_current_kernel_sources():
    # profiles/traffic.json holds the rocprofv3 FETCH_SIZE / WRITE_SIZE and pipe
    # counters that bench.py reports; each entry names the step kernels' source hash
    # it was taken with, and a stale entry is reported as null
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    sha = bench.kernel_source_sha()
    assert rec and all(v["source_sha"] == sha for v in rec.values()), \
        {k: v["source_sha"] for k, v in rec.items()}
    for key in rec:
        assert bench.measured_profile(key) == rec[key]

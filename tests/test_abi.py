"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every entry point declared in include/dgsn.h,
and do its host-only work (quadrature, descriptor validation, artifact
parsing) correctly.  No device call is made here.
"""
import ctypes
import json
import os
import re
import struct
import zlib

import numpy as np
import pytest

import oracle
from paper_1906_04017_amd import _lib, ann_format
from paper_1906_04017_amd._lib import ProblemDesc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1906_04017_amd import build
        build.build()
    return _lib.load()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "dgsn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dgsn_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_symbols()
    for required in ("dgsn_problem_create", "dgsn_sweep", "dgsn_source_iterate",
                     "dgsn_adjoint_solve", "dgsn_ann_load", "dgsn_ann_infer",
                     "dgsn_local_solve", "dgsn_batch_run"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(_lib.SIGNATURES)


def test_version(lib):
    assert lib.dgsn_version() >= 10000


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12])
def test_library_quadrature_matches_oracle(lib, order):
    from paper_1906_04017_amd import api
    om, w = api.quadrature_ls(order)
    om_o, w_o = oracle.lq_n(order)
    assert om.shape == om_o.shape
    # two independent root searches on an increasingly ill-conditioned
    # weight system (S10, S12): agreement to a few hundred ulps
    assert np.abs(om - om_o).max() < 1e-13
    assert np.abs(w - w_o).max() < 1e-13


def test_quadrature_rejects_bad_orders(lib):
    n = ctypes.c_int(0)
    for order in (0, 3, 14, -2):
        assert lib.dgsn_quadrature_ls(order, None, None, ctypes.byref(n)) == _lib.DGSN_EINVAL
    assert lib.dgsn_quadrature_ls(8, None, None, ctypes.byref(n)) == 0 and n.value == 80
    small = ctypes.c_int(10)
    om = np.zeros((80, 3))
    w = np.zeros(80)
    rc = lib.dgsn_quadrature_ls(8, om.ctypes.data_as(_lib._PD), w.ctypes.data_as(_lib._PD),
                                ctypes.byref(small))
    assert rc == _lib.DGSN_EINVAL and b"capacity" in lib.dgsn_last_error()


def _desc(**kw):
    om, w = oracle.lq_n(4)
    a = dict(n=(4, 4, 4), L=(1.0, 1.0, 1.0), G=1, om=om, w=w, prec=0, solver=0, store=0)
    a.update(kw)
    om = np.ascontiguousarray(a["om"], np.float64)
    w = np.ascontiguousarray(a["w"], np.float64)
    d = ProblemDesc(a["n"][0], a["n"][1], a["n"][2], a["L"][0], a["L"][1], a["L"][2], a["G"],
                    len(w), om.ctypes.data_as(_lib._PD), w.ctypes.data_as(_lib._PD), a["prec"],
                    a["solver"], a["store"])
    return d, (om, w)


def test_validation_accepts_good_descriptor(lib):
    d, keep = _desc()
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == 0


@pytest.mark.parametrize("kw,needle", [
    (dict(n=(0, 4, 4)), b"cells per axis"),
    (dict(n=(4, 4, 2000)), b"cells per axis"),
    (dict(L=(1.0, -1.0, 1.0)), b"domain length"),
    (dict(L=(1.0, float("nan"), 1.0)), b"domain length"),
    (dict(G=0), b"n_groups"),
    (dict(prec=7), b"precision"),
    (dict(solver=5), b"solver"),
    (dict(prec=1, solver=1), b"FP32"),
])
def test_validation_rejects_bad_descriptors(lib, kw, needle):
    d, keep = _desc(**kw)
    rc = lib.dgsn_problem_validate(ctypes.byref(d))
    assert rc in (_lib.DGSN_EINVAL, _lib.DGSN_EUNSUPPORTED)
    assert needle in lib.dgsn_last_error()


def test_validation_rejects_bad_quadratures(lib):
    om, w = oracle.lq_n(4)
    bad = om.copy()
    bad[3] *= 1.001
    d, keep = _desc(om=bad)
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == _lib.DGSN_EINVAL
    assert b"unit vector" in lib.dgsn_last_error()
    d, keep = _desc(w=w * 1.01)
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == _lib.DGSN_EINVAL
    assert b"4 pi" in lib.dgsn_last_error()
    w2 = w.copy()
    w2[0] = -w2[0]
    d, keep = _desc(w=w2)
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == _lib.DGSN_EINVAL
    # unbalanced octants: flip the sign of one direction
    om2 = om.copy()
    om2[0] = -om2[0]
    d, keep = _desc(om=om2)
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == _lib.DGSN_EINVAL
    assert b"octant" in lib.dgsn_last_error()
    d, keep = _desc(om=om[:20], w=w[:20] * 24 / 20)
    assert lib.dgsn_problem_validate(ctypes.byref(d)) == _lib.DGSN_EINVAL
    assert lib.dgsn_problem_validate(None) == _lib.DGSN_EINVAL


def test_null_handles_are_rejected(lib):
    assert lib.dgsn_sweep(None, None, None, None) == _lib.DGSN_EINVAL
    assert lib.dgsn_source_iterate(None, None, 1e-8, 10, None, None, None, None) == _lib.DGSN_EINVAL
    assert lib.dgsn_adjoint_solve(None, None, None, None, 1e-8, 10, None, None) == _lib.DGSN_EINVAL
    assert lib.dgsn_problem_set_inflow(None, None) == _lib.DGSN_EINVAL
    out = ctypes.c_void_p()
    d, keep = _desc()
    assert lib.dgsn_problem_create(None, ctypes.byref(d), ctypes.byref(out)) == _lib.DGSN_EINVAL
    assert lib.dgsn_local_solve(None, None, None, 10, 0, None) == _lib.DGSN_EINVAL
    n = ctypes.c_int(-1)
    assert lib.dgsn_problem_si_history(None, None, None, 0, ctypes.byref(n)) == _lib.DGSN_EINVAL


def test_spectral_radius_estimate():
    from paper_1906_04017_amd.api import spectral_radius
    # a geometric residual sequence has its ratio as the estimate, over any tail
    for rho in (0.3, 0.859, 0.957):
        r = 2.5 * rho ** np.arange(40)
        assert abs(spectral_radius(r) - rho) < 1e-12
        assert abs(spectral_radius(r, tail=0.1) - rho) < 1e-12
    # a transient that has died out does not bias the tail estimate
    k = np.arange(60)
    r = 0.9 ** k + 5.0 * 0.2 ** k
    assert abs(spectral_radius(r) - 0.9) < 1e-9
    # too short or a zero residual: no estimate
    assert spectral_radius([1.0, 0.5, 0.25]) is None
    assert spectral_radius([1.0, 0.5, 0.25, 0.0]) is None


def _artifact(tmp_path, nh=64, act=0, seed=0):
    rng = np.random.default_rng(seed)
    p = tmp_path / f"net_{nh}_{act}.dgsnann"
    ann_format.write(p, rng.normal(size=(nh, 24)), rng.normal(size=nh), rng.normal(size=(8, nh)),
                     rng.normal(size=8), activation=act)
    return p


def test_artifact_roundtrip(tmp_path):
    p = _artifact(tmp_path)
    net = ann_format.read(p)
    assert net["W1"].shape == (64, 24) and net["W2"].shape == (8, 64)
    raw = open(p, "rb").read()
    assert raw[:8] == b"DGSNANN1"
    assert struct.unpack("<I", raw[-4:])[0] == zlib.crc32(raw[:-4]) & 0xFFFFFFFF


def test_ann_load_checks_file_before_device(lib, tmp_path):
    out = ctypes.c_void_p()
    good = _artifact(tmp_path)
    # valid file, no context: the format passes, the missing context is reported
    assert lib.dgsn_ann_load(None, str(good).encode(), ctypes.byref(out)) == _lib.DGSN_EINVAL
    assert b"ctx" in lib.dgsn_last_error()
    raw = bytearray(open(good, "rb").read())
    bad = tmp_path / "bad_magic.dgsnann"
    bad.write_bytes(b"XXXXXXXX" + bytes(raw[8:]))
    assert lib.dgsn_ann_load(None, str(bad).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    flip = bytearray(raw)
    flip[100] ^= 0x40
    bad.write_bytes(bytes(flip))
    assert lib.dgsn_ann_load(None, str(bad).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    assert b"checksum" in lib.dgsn_last_error()
    bad.write_bytes(bytes(raw[:-10]))
    assert lib.dgsn_ann_load(None, str(bad).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    tanh = _artifact(tmp_path, act=1)
    assert lib.dgsn_ann_load(None, str(tanh).encode(), ctypes.byref(out)) == _lib.DGSN_EUNSUPPORTED
    wide = _artifact(tmp_path, nh=96)
    assert lib.dgsn_ann_load(None, str(wide).encode(), ctypes.byref(out)) == _lib.DGSN_EUNSUPPORTED
    missing = tmp_path / "nope.dgsnann"
    assert lib.dgsn_ann_load(None, str(missing).encode(), ctypes.byref(out)) == _lib.DGSN_EINVAL


def _paper_artifact(tmp_path, name="paper.dgsnann", nh=8, **kw):
    rng = np.random.default_rng(5)
    imin, imax = np.zeros(26), np.ones(26)
    imin[12:14] = -1.0
    p = tmp_path / name
    ann_format.write_paper(p, rng.normal(size=(8, nh, 26)), rng.normal(size=(8, nh)),
                           rng.normal(size=(8, 8, nh)), rng.normal(size=(8, 8)),
                           kw.pop("imin", imin), kw.pop("imax", imax), **kw)
    return p


def test_paper_artifact_roundtrip(tmp_path):
    p = _paper_artifact(tmp_path)
    net = ann_format.read(p)
    assert net["version"] == 2 and net["W1"].shape == (8, 8, 26) and net["W2"].shape == (8, 8, 8)
    assert abs(net["alpha"] - 0.27) < 1e-7 and abs(net["beta_scale"] - 0.1) < 1e-7
    raw = open(p, "rb").read()
    assert struct.unpack("<7I", raw[8:36]) == (2, 26, 8, 8, 1, 1, 8)


def test_paper_ann_load_checks_file_before_device(lib, tmp_path):
    out = ctypes.c_void_p()
    good = _paper_artifact(tmp_path)
    assert lib.dgsn_ann_load(None, str(good).encode(), ctypes.byref(out)) == _lib.DGSN_EINVAL
    assert b"ctx" in lib.dgsn_last_error()
    wide = _paper_artifact(tmp_path, "wide.dgsnann", nh=9)
    assert lib.dgsn_ann_load(None, str(wide).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    relu = _paper_artifact(tmp_path, "relu.dgsnann", activation=0)
    assert lib.dgsn_ann_load(None, str(relu).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    noelu = _paper_artifact(tmp_path, "noelu.dgsnann", flags=0)
    assert lib.dgsn_ann_load(None, str(noelu).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    flat = _paper_artifact(tmp_path, "flat.dgsnann", imin=np.ones(26), imax=np.ones(26))
    assert lib.dgsn_ann_load(None, str(flat).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    assert b"bounds" in lib.dgsn_last_error()
    raw = open(good, "rb").read()
    short = tmp_path / "short.dgsnann"
    short.write_bytes(raw[:60])
    assert lib.dgsn_ann_load(None, str(short).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    assert lib.dgsn_ann_infer_octant(None, 0, None, None, 1, None) == _lib.DGSN_EINVAL
    v = ctypes.c_int()
    assert lib.dgsn_ann_info(None, ctypes.byref(v), None, None, None) == _lib.DGSN_EINVAL


def _paper_dir_artifact(tmp_path, name="pdir.dgsnann", omega=None, nh=8):
    rng = np.random.default_rng(6)
    om = oracle.lq_n(4)[0] if omega is None else np.asarray(omega)
    k = len(om)
    imin, imax = np.zeros(26), np.ones(26)
    imin[12:14] = -1.0
    p = tmp_path / name
    ann_format.write_paper_dir(p, rng.normal(size=(k, nh, 26)), rng.normal(size=(k, nh)),
                               rng.normal(size=(k, 8, nh)), rng.normal(size=(k, 8)), imin, imax,
                               om)
    return p


def test_paper_dir_artifact_roundtrip_and_load_checks(lib, tmp_path):
    from oracle import ann_paper_train
    p = _paper_dir_artifact(tmp_path)
    net = ann_format.read(p)
    assert net["version"] == 3 and net["W1"].shape == (24, 8, 26) and net["omega"].shape == (24, 3)
    raw = open(p, "rb").read()
    assert struct.unpack("<7I", raw[8:36]) == (3, 26, 8, 8, 1, 1, 24)
    # the oracle's reader sees the same networks and directions
    o = ann_paper_train.read_artifact(p)
    assert np.array_equal(o["W1"], net["W1"].astype(np.float64))
    assert np.array_equal(o["omega"], net["omega"].astype(np.float64))
    out = ctypes.c_void_p()
    assert lib.dgsn_ann_load(None, str(p).encode(), ctypes.byref(out)) == _lib.DGSN_EINVAL
    assert b"ctx" in lib.dgsn_last_error()
    om = oracle.lq_n(4)[0].copy()
    om[3] *= 1.01
    bad = _paper_dir_artifact(tmp_path, "norm.dgsnann", omega=om)
    assert lib.dgsn_ann_load(None, str(bad).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    assert b"unit" in lib.dgsn_last_error()
    om = oracle.lq_n(4)[0].copy()
    om[5] = om[2]
    dup = _paper_dir_artifact(tmp_path, "dup.dgsnann", omega=om)
    assert lib.dgsn_ann_load(None, str(dup).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT
    assert b"coincide" in lib.dgsn_last_error()
    short = tmp_path / "short_dir.dgsnann"
    short.write_bytes(raw[:44 + 8 * 26 + 40])
    assert lib.dgsn_ann_load(None, str(short).encode(), ctypes.byref(out)) == _lib.DGSN_EFORMAT


@pytest.mark.parametrize("name", ["sigma10_h0.078125", "sigma0.001_h0.078125", "sigma10_h0.1",
                                  "sigma0.001_h0.1", "sigma10_h0.078125_psi12_s120",
                                  "sigma10_h0.1_psi12_s120"])
def test_trained_per_direction_artifacts(name):
    # the shipped per-direction networks: one 26-8-8 network for each of the
    # 80 LQ_8 directions, stored with the direction it serves; the input
    # bounds are the training ranges (inflow and source maxima)
    from oracle import ann_paper_train
    path = os.path.join(ROOT, "paper_1906_04017_amd", "data", f"ann_paper_dir_s8_{name}.dgsnann")
    net = ann_paper_train.read_artifact(path)
    om, _ = oracle.lq_n(8)
    assert net["W1"].shape == (80, 8, 26) and net["W2"].shape == (80, 8, 8)
    assert np.abs(net["omega"] - om).max() < 1e-6
    psi_max, s_max = (12.0, 120.0) if name.endswith("_psi12_s120") else (1.0, 1.0)
    assert np.all(net["imax"][:12] == psi_max) and np.all(net["imax"][14:22] == s_max)


def test_trained_paper_artifact_shape():
    # the shipped paper-form artifact: 8 octant networks of 26-8-8 with at most
    # the paper's 272 connections each (Sec. 3; fewer after pruning)
    from oracle import ann_paper_train
    path = os.path.join(ROOT, "paper_1906_04017_amd", "data", "ann_paper_tanh8.dgsnann")
    net = ann_paper_train.read_artifact(path)
    assert net["W1"].shape == (8, 8, 26) and net["W2"].shape == (8, 8, 8)
    for o in range(8):
        conn = int(np.count_nonzero(net["W1"][o]) + np.count_nonzero(net["W2"][o]))
        assert 0 < conn <= 26 * 8 + 8 * 8
    assert abs(net["alpha"] - 0.27) < 1e-6 and abs(net["beta_scale"] - 0.1) < 1e-6


def test_library_harmonics_match_oracle(lib):
    from paper_1906_04017_amd import api
    rng = np.random.default_rng(140)
    om = rng.normal(size=(25, 3))
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    om = np.concatenate([om, oracle.lq_n(8)[0]])
    for L in range(4):
        assert np.abs(api.real_ylm(L, om) - oracle.real_ylm(L, om)).max() < 1e-14
    with pytest.raises(api.DgsnError):
        api.real_ylm(4, om)


def test_autotune_cache_file_roundtrip(lib, tmp_path):
    # the autotuner cache is host state: a file written by hand loads, saves
    # back with the same entries, and malformed files leave it unchanged
    from paper_1906_04017_amd import api
    api.autotune_cache_clear()
    assert api.autotune_cache_size() == 0
    src = tmp_path / "tune.json"
    src.write_text('{"dgsn_autotune_cache": 1, "entries": [\n'
                   '  {"key": "shape-a", "tile": 2, "schedule": 1, "ms": [1.5, 1.25, 2, -1, 1.125, 3]},\n'
                   '  {"key": "shape-b", "tile": 3, "schedule": 0, "ms": [4, 3.5, 3, -1, -1, -1]}\n'
                   ']}\n')
    api.autotune_cache_load(src)
    assert api.autotune_cache_size() == 2
    out = tmp_path / "out.json"
    api.autotune_cache_save(out)
    lines = [l.strip() for l in out.read_text().splitlines()]
    assert lines[0].startswith('{"dgsn_autotune_cache": 1')
    assert '{"key": "shape-a", "tile": 2, "schedule": 1, "ms": [1.5, 1.25, 2, -1, 1.125, 3]},' in lines
    assert '{"key": "shape-b", "tile": 3, "schedule": 0, "ms": [4, 3.5, 3, -1, -1, -1]}' in lines
    json.loads(out.read_text())   # a JSON document
    bad = tmp_path / "bad.json"
    bad.write_text('{"dgsn_autotune_cache": 1, "entries": [\n'
                   '  {"key": "shape-c", "tile": 7, "schedule": 0, "ms": [1, 1, 1, 1, 1, 1]}\n]}\n')
    with pytest.raises(api.DgsnError, match="EFORMAT"):
        api.autotune_cache_load(bad)
    other = tmp_path / "other.json"
    other.write_text('{"entries": []}\n')
    with pytest.raises(api.DgsnError, match="EFORMAT"):
        api.autotune_cache_load(other)
    with pytest.raises(api.DgsnError, match="EINVAL"):
        api.autotune_cache_load(tmp_path / "missing.json")
    assert api.autotune_cache_size() == 2
    api.autotune_cache_clear()
    assert api.autotune_cache_size() == 0

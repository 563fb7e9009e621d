"""GPU parity of the HIP transport path against the FP64 CPU oracle.

Every device call goes through the C ABI (paper_1906_04017_amd.api is plain
ctypes marshalling).  Both sides get the same seeded inputs from
paper_1906_04017_amd.inputs; the GPU uses the library's own LQ_N quadrature,
the oracle its own independent construction (they agree to 1e-13).

Tolerances (norm-wise relative error max|a - b| / max|b| unless stated):
  FP64 sweep / SI / adjoint  1e-12 / 1e-10 / 1e-10  (rounding only; different
                             assembly order and element-matrix construction)
  FP32 sweep and SI          1e-5   (the stated FP32 GE target)
  FP32 adjoint gradients     1e-4
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1906_04017_amd import inputs

pytestmark = pytest.mark.gpu

FP64_SWEEP_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def api():
    from paper_1906_04017_amd import api as _api
    return _api


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def mesh_of(p):
    return (*p["n"], *p["length"])


def gpu_problem(api, ctx, p, precision, solver="ge", store_psi=False):
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision=precision,
                       solver=solver, store_psi=store_psi)
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    return prob


def nodal_source(p, seed=None):
    """q as a nodal field, plus an optional random nodal part."""
    S = np.repeat(p["q"][..., None], 8, axis=-1)
    if seed is not None:
        S = S + inputs.random_nodal(p["sigma_t"].shape[1], p["groups"], seed, -0.2, 0.5)
    return S


def print_case(case, **kw):
    print(f"[case] {case} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


# ---------------------------------------------------------------------------
# one-cell GE
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_local_solve_matches_oracle(api, ctx, precision, tol):
    print_case("local_solve", precision=precision)
    rng = np.random.default_rng(101)
    n = 4099
    om = np.abs(rng.normal(size=(n, 3)))
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    h = rng.uniform(0.2, 2.0, size=(n, 3))
    st = 10 ** rng.uniform(-4, 1.3, size=n)
    S = rng.uniform(-0.1, 1.0, size=(n, 8))
    pin = rng.uniform(-0.1, 1.0, size=(n, 12))
    up = np.zeros((n, 6, 8))
    for fn in range(4):
        up[:, 0, 2 * fn] = pin[:, fn]
        up[:, 2, (fn & 1) + 4 * (fn >> 1)] = pin[:, 4 + fn]
        up[:, 4, fn] = pin[:, 8 + fn]
    ref = oracle.cell_solve_batch(h, om, st, S, up)
    hh = np.cbrt(h.prod(axis=1))
    x = np.concatenate([om * hh[:, None] / h, (st * hh)[:, None], pin, S * hh[:, None]], axis=1)
    dt = torch.float64 if precision == "fp64" else torch.float32
    y = api.local_solve(ctx, torch.tensor(x, dtype=dt, device="cuda")).cpu().numpy()
    err = np.abs(y - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() < tol


# ---------------------------------------------------------------------------
# sweep
# ---------------------------------------------------------------------------

def test_sweep_absorber_cube_fp64(api, ctx):
    p = inputs.absorber_cube()
    print_case("sweep", name=p["name"], precision="fp64")
    prob = gpu_problem(api, ctx, p, "fp64")
    S = nodal_source(p)
    phi = prob.sweep(torch.tensor(S, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(p["order"])
    ref = oracle.sweep(mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= FP64_SWEEP_TOL


RAGGED = [
    ((1, 1, 1), (0.3, 0.3, 0.3), 2, 1),
    ((5, 3, 2), (1.0, 0.6, 0.5), 4, 3),
    ((7, 2, 9), (0.7, 0.2, 1.8), 6, 2),
    ((4, 6, 3), (1.0, 1.5, 0.75), 12, 1),
    ((9, 9, 9), (1.0, 1.0, 1.0), 8, 5),
]


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("solver", ["ge", "ge_dense"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", RAGGED, ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in RAGGED])
def test_sweep_ragged_meshes(api, ctx, precision, case, solver, tile):
    n, L, order, G = case
    print_case("sweep", n=n, order=order, G=G, precision=precision, solver=solver, tile=tile)
    p = inputs.random_problem(n, order, G, seed=hash(case) % 1000, length=L)
    prob = gpu_problem(api, ctx, p, precision, solver=solver)
    prob.set_tile(tile)
    S = nodal_source(p, seed=7)
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi = prob.sweep(torch.tensor(S, dtype=dt, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(order)
    ref = oracle.sweep(mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= (FP64_SWEEP_TOL if precision == "fp64" else FP32_TOL)


def test_sweep_multi_group_multi_tile(api, ctx):
    # several blocks per hyperplane and a ragged last block (Do = 10, G = 7)
    p = inputs.random_problem((12, 10, 11), 8, 7, seed=5, length=(1.2, 1.0, 1.1))
    print_case("sweep", name=p["name"], precision="fp32")
    prob = gpu_problem(api, ctx, p, "fp32")
    S = nodal_source(p, seed=9)
    phi = prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(8)
    ref = oracle.sweep(mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= FP32_TOL


def test_sweep_is_deterministic(api, ctx):
    p = inputs.random_problem((10, 9, 8), 6, 3, seed=11)
    print_case("determinism", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32")
    S = torch.tensor(nodal_source(p, seed=3), dtype=torch.float32, device="cuda")
    a = prob.sweep(S).cpu()
    b = prob.sweep(S).cpu()
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 3e-6)])
def test_constant_solution_invariant(api, ctx, precision, tol):
    # uniform sigma_t and q with matching inflow q/sigma_t on every face:
    # psi == q/sigma_t at every node, so phi == 4 pi q / sigma_t
    n = (6, 5, 7)
    print_case("constant_solution", n=n, precision=precision)
    ncell = 6 * 5 * 7
    st, qv = 3.3, 1.7
    p = inputs.problem(n, (0.6, 0.5, 0.9), 8, 2, np.full((2, ncell), st), np.zeros((2, ncell)),
                       np.full((2, ncell), qv), np.full(6, qv / st), "const")
    prob = gpu_problem(api, ctx, p, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi = prob.sweep(torch.full((2, ncell, 8), qv, dtype=dt, device="cuda")).cpu().numpy()
    assert np.abs(phi / (4 * np.pi * qv / st) - 1).max() < tol


# ---------------------------------------------------------------------------
# source iteration
# ---------------------------------------------------------------------------

def test_source_iteration_fp64(api, ctx):
    p = inputs.random_problem((6, 5, 4), 4, 2, seed=21, c_max=0.8)
    print_case("source_iterate", name=p["name"], precision="fp64")
    prob = gpu_problem(api, ctx, p, "fp64")
    phi, info = prob.source_iterate(tol=1e-13, max_iter=500)
    om, w = oracle.lq_n(4)
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-14, max_iter=1000)
    assert info["converged"] and ref["converged"]
    assert rel(phi.cpu().numpy(), ref["phi"]) <= 1e-10


def test_source_iteration_fp32_blocky(api, ctx):
    p = inputs.blocky_scatter(n=16, groups=3, seed=2, order=8)
    print_case("source_iterate", name=p["name"], precision="fp32")
    prob = gpu_problem(api, ctx, p, "fp32")
    phi, info = prob.source_iterate(tol=1e-8, max_iter=400, allow_notconv=True)
    om, w = oracle.lq_n(8)
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-12, max_iter=2000)
    assert ref["converged"]
    assert info["resid"] < 1e-6
    for g in range(p["groups"]):
        assert rel(phi.cpu().numpy()[g], ref["phi"][g]) <= FP32_TOL


def test_source_iteration_resume_from_saved_phi(api, ctx):
    p = inputs.random_problem((5, 5, 5), 4, 1, seed=23, c_max=0.9)
    print_case("source_iterate_resume", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp64")
    full, info_full = prob.source_iterate(tol=1e-12, max_iter=1000)
    part, info_part = prob.source_iterate(tol=1e-12, max_iter=5, allow_notconv=True)
    assert not info_part["converged"] and info_part["iters"] == 5
    rest, info_rest = prob.source_iterate(phi0=part, tol=1e-12, max_iter=1000)
    assert info_rest["converged"]
    assert rel(rest.cpu().numpy(), full.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("precision,schedule", [("fp32", "dataflow"), ("fp32", "planes"),
                                                 ("fp64", "planes")])
def test_overlapped_iteration_equals_serial(api, ctx, precision, schedule):
    # source iteration overlaps each sweep with the previous residual
    # readback on alternating iterate buffers; a problem that stores psi
    # iterates serially in place.  Both must give the same iterates, residuals
    # and counts, for stops at odd and even iteration counts.
    p = inputs.blocky_scatter(n=12, groups=3, seed=5, order=4)
    print_case("overlapped_si", name=p["name"], precision=precision, schedule=schedule)
    a = gpu_problem(api, ctx, p, precision)
    b = gpu_problem(api, ctx, p, precision, store_psi=True)
    for prob in (a, b):
        prob.set_schedule(schedule)
        prob.set_si_criterion("fixed")
    for k in (1, 2, 3, 6):
        pa, ia = a.source_iterate(tol=0.0, max_iter=k)
        pb, ib = b.source_iterate(tol=0.0, max_iter=k)
        assert ia["iters"] == ib["iters"] == k
        assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy()), k
        assert np.array_equal(a.si_history()[0], b.si_history()[0])
    # stopping by the tolerance
    for prob in (a, b):
        prob.set_si_criterion("maxnorm")
    tol = 1e-5 if precision == "fp32" else 1e-9
    pa, ia = a.source_iterate(tol=tol, max_iter=500, allow_notconv=True)
    pb, ib = b.source_iterate(tol=tol, max_iter=500, allow_notconv=True)
    assert ia["iters"] == ib["iters"] and ia["resid"] == ib["resid"]
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
    # the kernel timing covers every sweep of the call
    a.set_timing(True)
    a.set_si_criterion("fixed")
    a.source_iterate(tol=0.0, max_iter=4)
    ms, launches = a.kernel_time()
    assert ms > 0 and launches >= 4 and launches % 4 == 0
    assert schedule != "dataflow" or launches == 4
    a.set_timing(False)


def test_source_iteration_history_matches_oracle_steps(api, ctx):
    """The recorded residual and eps_S of every iteration equal the oracle's
    after one step from the same iterate, and the effective spectral radius
    they give lies below the largest scattering ratio."""
    p = inputs.random_problem((5, 4, 4), 4, 2, seed=25, c_max=0.9)
    print_case("source_iterate_history", name=p["name"], precision="fp64")
    prob = gpu_problem(api, ctx, p, "fp64")
    assert prob.si_history()[0].size == 0
    phi, info = prob.source_iterate(tol=1e-11, max_iter=500)
    r, e = prob.si_history()
    assert info["converged"] and r.size == e.size == info["iters"]
    assert r[-1] == info["resid"] and e[-1] == info["eps_s"]
    om, w = oracle.lq_n(4)
    ph, ref_r, ref_e = None, [], []
    for _ in range(12):
        out = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                    p["psi_inc"], tol=0.0, max_iter=1, phi0=ph)
        ref_r.append(out["resid"])
        ref_e.append(out["eps_s"])
        ph = out["phi"]
    np.testing.assert_allclose(r[:12], ref_r, rtol=1e-9)
    np.testing.assert_allclose(e[:12], ref_e, rtol=1e-9)
    rho = api.spectral_radius(r)
    c = (p["sigma_s"] / p["sigma_t"]).max()
    assert rho is not None and 0.0 < rho < c
    # a second call replaces the history
    prob.source_iterate(phi0=phi, tol=1e-11, max_iter=500)
    assert prob.si_history()[0].size <= 2


# ---------------------------------------------------------------------------
# anisotropic in-group P_L scattering
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,L", [("fp64", 1), ("fp64", 2), ("fp64", 3), ("fp32", 1),
                                         ("fp32", 3)])
def test_pl_source_iteration_matches_oracle(api, ctx, precision, L):
    p = inputs.random_problem((6, 5, 4), 4, 2, seed=110 + L, c_max=0.8,
                              length=(0.6, 0.5, 0.4))
    sn = inputs.anisotropic_orders(p["sigma_s"], L, seed=120 + L)
    print_case("pl_si", name=p["name"], precision=precision, L=L)
    prob = gpu_problem(api, ctx, p, precision)
    prob.set_anisotropy(sn)
    tol = 1e-13 if precision == "fp64" else 1e-8
    phi, info = prob.source_iterate(tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    mom = prob.moments().double().cpu().numpy()
    om, w = oracle.lq_n(4)
    ref = oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"],
                                   np.concatenate([p["sigma_s"][None], sn]), p["q"], p["psi_inc"],
                                   tol=1e-14, max_iter=3000)
    assert ref["converged"]
    bound = 1e-10 if precision == "fp64" else FP32_TOL
    assert rel(phi.cpu().numpy(), ref["phi"]) <= bound
    assert mom.shape == ref["mom"].shape
    scale = np.abs(ref["phi"]).max()
    assert np.abs(mom - ref["mom"]).max() <= bound * scale
    # the anisotropy is felt: the isotropic iteration differs
    iso = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-14, max_iter=3000)
    assert rel(iso["phi"], ref["phi"]) > 100 * bound


@pytest.mark.parametrize("order,L,gg", [(6, 1, False), (6, 2, False), (8, 3, False),
                                        (8, 2, True), (12, 3, False)])
def test_pl_staged_sources_fp32_match_oracle(api, ctx, order, L, gg):
    # FP32 sweeps with 8 or more moments and 6 or more directions per octant
    # stage each cell's moment sources in LDS once per direction segment
    # (L = 2, 3 at S8 and S12 here; L = 1 and S4 load them per lane):
    # source iteration against the oracle
    p = inputs.random_problem((5, 4, 6), order, 2, seed=240 + order + L, c_max=0.7,
                              length=(0.5, 0.4, 0.6))
    print_case("pl_staged", name=p["name"], L=L, gg=gg)
    prob = gpu_problem(api, ctx, p, "fp32")
    om, w = oracle.lq_n(order)
    if gg:
        sn = _multigroup_pl(p, L, 250 + L)
        prob.set_anisotropy_gg(sn)
        full = sn
    else:
        sn = inputs.anisotropic_orders(p["sigma_s"], L, seed=250 + L)
        prob.set_anisotropy(sn)
        full = np.concatenate([p["sigma_s"][None], sn])
    for sched in ("planes", "dataflow"):
        prob.set_schedule(sched)
        phi, info = prob.source_iterate(tol=1e-8, max_iter=1000, allow_notconv=True)
        mom = prob.moments().double().cpu().numpy()
        ref = oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"], full, p["q"],
                                       p["psi_inc"], tol=1e-14, max_iter=3000, gg=gg)
        assert ref["converged"]
        for g in range(p["groups"]):
            assert rel(phi.cpu().numpy()[g], ref["phi"][g]) <= FP32_TOL, (sched, g)
        assert np.abs(mom - ref["mom"]).max() <= FP32_TOL * np.abs(ref["phi"]).max(), sched


@pytest.mark.parametrize("L", [2, 3])
def test_pl_staged_sources_fp32_adjoint(api, ctx, L):
    p = inputs.random_problem((4, 5, 4), 8, 2, seed=260 + L, c_max=0.7,
                              length=(0.4, 0.5, 0.4))
    sn = inputs.anisotropic_orders(p["sigma_s"], L, seed=265 + L)
    print_case("pl_staged_adjoint", name=p["name"], L=L)
    prob = gpu_problem(api, ctx, p, "fp32", store_psi=True)
    prob.set_anisotropy(sn)
    prob.source_iterate(tol=1e-7, max_iter=1000, allow_notconv=True)
    rng = np.random.default_rng(270 + L)
    g = rng.uniform(0.0, 1.0, (2, p["sigma_t"].shape[1], 8))
    gst, gq, info = prob.adjoint(g, tol=1e-7, max_iter=1000, allow_notconv=True)
    om, w = oracle.lq_n(8)
    full = np.concatenate([p["sigma_s"][None], sn])
    r = oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"], full, p["q"], p["psi_inc"],
                                 tol=1e-15, max_iter=3000, store_psi=True)
    a = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], r["psi"], r["phi"], g,
                       tol=1e-15, sigma_sn=full)
    assert rel(gst.cpu().numpy(), a["grad_sigma_t"]) <= 1e-4
    assert rel(gq.cpu().numpy(), a["grad_q"]) <= 1e-4


def test_pl_schedules_and_tiles_bitwise(api, ctx):
    p = inputs.random_problem((7, 6, 5), 8, 2, seed=130, c_max=0.7)
    sn = inputs.anisotropic_orders(p["sigma_s"], 2, seed=131)
    print_case("pl_schedules", name=p["name"])
    out = {}
    for sched in ("planes", "dataflow"):
        for b in (1, 2, 3):
            prob = gpu_problem(api, ctx, p, "fp32")
            prob.set_anisotropy(sn)
            prob.set_schedule(sched)
            prob.set_tile(b)
            phi, _ = prob.source_iterate(tol=0.0, max_iter=6, allow_notconv=True)
            out[(sched, b)] = (phi.cpu().numpy(), prob.moments().cpu().numpy())
            prob.close()
    for b in (1, 2, 3):
        assert np.array_equal(out[("planes", b)][0], out[("dataflow", b)][0])
        assert np.array_equal(out[("planes", b)][1], out[("dataflow", b)][1])
    # tile edges differ only by the rounding of the solve order within a tile
    assert rel(out[("planes", 2)][0], out[("planes", 1)][0]) <= FP32_TOL


def test_pl_zero_orders_equal_isotropic_bitwise(api, ctx):
    p = inputs.random_problem((5, 5, 4), 4, 2, seed=132, c_max=0.8)
    print_case("pl_zero_orders", name=p["name"])
    a = gpu_problem(api, ctx, p, "fp64")
    phi_a, ia = a.source_iterate(tol=1e-12, max_iter=500)
    b = gpu_problem(api, ctx, p, "fp64")
    b.set_anisotropy(np.zeros((3, 2, p["sigma_t"].shape[1])))
    phi_b, ib = b.source_iterate(tol=1e-12, max_iter=500)
    assert ia["iters"] == ib["iters"]
    assert np.array_equal(phi_a.cpu().numpy(), phi_b.cpu().numpy())
    # the moments are those of the (anisotropic) angular flux itself, here
    # of the isotropic-scattering solution: sum_d w_d Y_k(Omega_d) psi_d
    om, w = oracle.lq_n(4)
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-14, max_iter=3000, store_psi=True)
    Y = oracle.real_ylm(3, om)
    mom_ref = np.einsum("d,dk,dgcn->kgcn", w, Y[:, 1:], ref["psi"])
    assert np.abs(b.moments().cpu().numpy() - mom_ref).max() <= 1e-10 * np.abs(ref["phi"]).max()
    assert np.abs(mom_ref).max() > 1e-3 * np.abs(ref["phi"]).max()
    # removing the orders restores the isotropic problem
    b.set_anisotropy(None)
    phi_c, _ = b.source_iterate(tol=1e-12, max_iter=500)
    assert np.array_equal(phi_a.cpu().numpy(), phi_c.cpu().numpy())


def test_pl_constant_solution(api, ctx):
    # uniform medium, inflow c on every face, q = (sigma_t - sigma_s0) c:
    # psi == c, and every moment of the constant flux vanishes for the
    # level-symmetric set, so the anisotropic orders leave it unchanged
    n = (6, 5, 4)
    nc = 120
    cval = 0.7
    st = np.full((1, nc), 2.0)
    ss = np.full((1, nc), 1.2)
    p = inputs.problem(n, (0.6, 0.5, 0.4), 6, 1, st, ss, cval * (st - ss), np.full(6, cval),
                       "pl_constant")
    print_case("pl_constant", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp64")
    prob.set_anisotropy(np.stack([np.full((1, nc), v) for v in (0.6, 0.3, 0.15)]))
    phi, info = prob.source_iterate(tol=1e-14, max_iter=2000)
    assert np.abs(phi.cpu().numpy() / (4 * np.pi) - cval).max() < 1e-12
    assert prob.moments().abs().max().item() < 1e-12


def test_pl_rejections(api, ctx):
    p = inputs.random_problem((3, 3, 3), 4, 2, seed=133, c_max=0.5)
    prob = gpu_problem(api, ctx, p, "fp32", solver="ge_dense", store_psi=True)
    sn = inputs.anisotropic_orders(p["sigma_s"], 1, seed=134)
    with pytest.raises(api.DgsnError, match="EINVAL"):
        prob.moments()
    with pytest.raises(api.DgsnError, match="EINVAL"):
        prob.set_anisotropy(np.zeros((4, 2, 27)))
    prob.set_anisotropy(sn)
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.set_scattering(np.zeros((2, 2, 27)))
    # the psi store and the adjoint take the mass-inverse form
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.source_iterate(tol=1e-6, max_iter=200, allow_notconv=True)
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.adjoint(np.ones((2, 27, 8)))
    prob.set_anisotropy(None)
    prob.set_scattering(np.zeros((2, 2, 27)))
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.set_anisotropy(sn)


@pytest.mark.parametrize("precision,L", [("fp64", 1), ("fp64", 2), ("fp32", 1), ("fp32", 3)])
def test_pl_adjoint_matches_oracle(api, ctx, precision, L):
    p = inputs.random_problem((5, 4, 4), 4, 2, seed=140 + L, c_max=0.7,
                              length=(0.5, 0.4, 0.4))
    sn = inputs.anisotropic_orders(p["sigma_s"], L, seed=150 + L)
    print_case("pl_adjoint", name=p["name"], precision=precision, L=L)
    prob = gpu_problem(api, ctx, p, precision, store_psi=True)
    prob.set_anisotropy(sn)
    tol = 1e-13 if precision == "fp64" else 1e-7
    prob.source_iterate(tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    rng = np.random.default_rng(160 + L)
    g = rng.uniform(0.0, 1.0, (2, p["sigma_t"].shape[1], 8))
    gst, gq, info = prob.adjoint(g, tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    om, w = oracle.lq_n(4)
    full = np.concatenate([p["sigma_s"][None], sn])
    r = oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"], full, p["q"], p["psi_inc"],
                                 tol=1e-15, max_iter=3000, store_psi=True)
    a = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], r["psi"], r["phi"], g,
                       tol=1e-15, sigma_sn=full)
    bound = 1e-9 if precision == "fp64" else 1e-4
    assert rel(gst.cpu().numpy(), a["grad_sigma_t"]) <= bound
    assert rel(gq.cpu().numpy(), a["grad_q"]) <= bound
    # the anisotropy is felt in the gradients
    iso = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], r["psi"], r["phi"], g,
                         tol=1e-15)
    assert rel(iso["grad_q"], a["grad_q"]) > 100 * bound


# ---------------------------------------------------------------------------
# multigroup scattering (group-to-group matrix, P0)
# ---------------------------------------------------------------------------

def _multigroup(p, seed, up=0.05, c=0.8):
    """Group-to-group matrix [G, G, ncell] (from g' into g): downscatter and
    in-group terms, a little upscatter, total scattering c sigma_t per group."""
    rng = np.random.default_rng(seed)
    G, nc = p["sigma_t"].shape
    gg = rng.uniform(0.0, 1.0, (G, G, nc))
    for g2 in range(G):
        for g in range(g2):
            gg[g2, g] *= up
    return gg * (c * p["sigma_t"])[None] / gg.sum(axis=0, keepdims=True)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", FP32_TOL)])
def test_multigroup_source_iteration_matches_oracle(api, ctx, precision, tol):
    p = inputs.random_problem((6, 5, 4), 4, 3, seed=81, length=(0.6, 0.5, 0.4))
    gg = _multigroup(p, 82)
    print_case("multigroup_si", name=p["name"], precision=precision)
    prob = gpu_problem(api, ctx, p, precision)
    prob.set_scattering(gg)
    si_tol = 1e-13 if precision == "fp64" else 1e-8
    phi, info = prob.source_iterate(tol=si_tol, max_iter=1000, allow_notconv=precision == "fp32")
    om, w = oracle.lq_n(4)
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], np.zeros_like(p["sigma_t"]),
                                p["q"], p["psi_inc"], tol=1e-14, max_iter=3000, sigma_gg=gg)
    assert ref["converged"]
    for g in range(p["groups"]):
        assert rel(phi.cpu().numpy()[g], ref["phi"][g]) <= tol, g
    # removing the matrix returns to the in-group sigma_s of set_materials
    prob.set_scattering(None)
    phi0, _ = prob.source_iterate(tol=si_tol, max_iter=1000, allow_notconv=precision == "fp32")
    ref0 = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                 p["psi_inc"], tol=1e-14, max_iter=3000)
    assert rel(phi0.cpu().numpy(), ref0["phi"]) <= tol


def test_multigroup_diagonal_matrix_is_in_group_scattering(api, ctx):
    p = inputs.random_problem((5, 4, 4), 4, 2, seed=83, c_max=0.8)
    print_case("multigroup_diag", name=p["name"])
    diag = np.zeros((2, 2, p["sigma_t"].shape[1]))
    for g in range(2):
        diag[g, g] = p["sigma_s"][g]
    prob = gpu_problem(api, ctx, p, "fp64")
    a, ia = prob.source_iterate(tol=1e-12, max_iter=1000)
    prob.set_scattering(diag)
    b, ib = prob.source_iterate(tol=1e-12, max_iter=1000)
    assert ia["iters"] == ib["iters"]
    assert rel(b.cpu().numpy(), a.cpu().numpy()) <= 1e-14


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_multigroup_adjoint_matches_oracle(api, ctx, precision, tol):
    p = inputs.adjoint_box(n=6, groups=3, seed=84, box=(1, 4))
    gg = _multigroup(p, 85, c=0.6)
    print_case("multigroup_adjoint", name=p["name"], precision=precision)
    prob = gpu_problem(api, ctx, p, precision, store_psi=True)
    prob.set_scattering(gg)
    si_tol = 1e-13 if precision == "fp64" else 1e-7
    prob.source_iterate(tol=si_tol, max_iter=1000, allow_notconv=True)
    nc = p["sigma_t"].shape[1]
    g = np.zeros((p["groups"], nc, 8))
    g[:, p["box_mask"], :] = 1.0
    dt = torch.float64 if precision == "fp64" else torch.float32
    gst, gq, _ = prob.adjoint(torch.tensor(g, dtype=dt, device="cuda"), tol=si_tol,
                              max_iter=1000, allow_notconv=True)
    om, w = oracle.lq_n(p["order"])
    zero = np.zeros_like(p["sigma_t"])
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], zero, p["q"], p["psi_inc"],
                                tol=1e-14, max_iter=3000, store_psi=True, sigma_gg=gg)
    a = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], zero, ref["psi"], ref["phi"], g,
                       tol=1e-14, sigma_gg=gg)
    assert rel(gst.cpu().numpy(), a["grad_sigma_t"]) <= tol
    assert rel(gq.cpu().numpy(), a["grad_q"]) <= tol


# ---------------------------------------------------------------------------
# anisotropic scattering with a group-to-group matrix per Legendre order
# ---------------------------------------------------------------------------

def _multigroup_pl(p, L, seed, c=0.8, ratios=(0.5, 0.25, 0.12)):
    """[L+1, G, G, ncell] (from g' into g at [n, g', g]): the order-0 matrix
    of _multigroup and forward-peaked higher orders r_n u sigma_0(g' -> g)."""
    rng = np.random.default_rng(seed + 1000)
    gg = _multigroup(p, seed, c=c)
    return np.stack([gg] + [ratios[n] * rng.uniform(0.8, 1.0, gg.shape) * gg for n in range(L)])


def _pl_gg_reference(p, sn, store_psi=False):
    om, w = oracle.lq_n(p["order"])
    return oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"], sn, p["q"], p["psi_inc"],
                                    tol=1e-14, max_iter=3000, gg=True, store_psi=store_psi)


@pytest.mark.parametrize("precision,L", [("fp64", 1), ("fp64", 2), ("fp64", 3), ("fp32", 2)])
def test_pl_gg_source_iteration_matches_oracle(api, ctx, precision, L):
    p = inputs.random_problem((6, 5, 4), 4, 3, seed=190 + L, length=(0.6, 0.5, 0.4))
    sn = _multigroup_pl(p, L, 195 + L)
    print_case("pl_gg_si", name=p["name"], precision=precision, L=L)
    prob = gpu_problem(api, ctx, p, precision)
    prob.set_anisotropy_gg(sn)
    tol = 1e-13 if precision == "fp64" else 1e-8
    phi, info = prob.source_iterate(tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    mom = prob.moments().double().cpu().numpy()
    ref = _pl_gg_reference(p, sn)
    assert ref["converged"]
    bound = 1e-10 if precision == "fp64" else FP32_TOL
    for g in range(p["groups"]):
        assert rel(phi.cpu().numpy()[g], ref["phi"][g]) <= bound, g
    assert mom.shape == ref["mom"].shape
    assert np.abs(mom - ref["mom"]).max() <= bound * np.abs(ref["phi"]).max()
    # the higher orders couple the groups: the in-group iteration of the
    # matrices' diagonals, with the same order-0 matrix, differs
    om, w = oracle.lq_n(p["order"])
    diag = sn.copy()
    for g2 in range(p["groups"]):
        for g in range(p["groups"]):
            if g != g2:
                diag[1:, g2, g] = 0.0
    alt = oracle.source_iterate_pl(mesh_of(p), om, w, p["sigma_t"], diag, p["q"], p["psi_inc"],
                                   tol=1e-14, max_iter=3000, gg=True)
    assert rel(alt["phi"], ref["phi"]) > 100 * bound


def test_pl_gg_schedules_and_tiles_bitwise(api, ctx):
    p = inputs.random_problem((7, 6, 5), 4, 3, seed=200)
    sn = _multigroup_pl(p, 2, 201)
    print_case("pl_gg_schedules", name=p["name"])
    out = {}
    for sched in ("planes", "dataflow"):
        for b in (1, 2):
            prob = gpu_problem(api, ctx, p, "fp32")
            prob.set_anisotropy_gg(sn)
            prob.set_schedule(sched)
            prob.set_tile(b)
            phi, _ = prob.source_iterate(tol=0.0, max_iter=6, allow_notconv=True)
            out[(sched, b)] = (phi.cpu().numpy(), prob.moments().cpu().numpy())
            prob.close()
    for b in (1, 2):
        assert np.array_equal(out[("planes", b)][0], out[("dataflow", b)][0])
        assert np.array_equal(out[("planes", b)][1], out[("dataflow", b)][1])
    assert rel(out[("planes", 2)][0], out[("planes", 1)][0]) <= FP32_TOL


def test_pl_gg_diagonal_matrices_equal_in_group(api, ctx):
    p = inputs.random_problem((5, 4, 4), 4, 2, seed=202, c_max=0.8)
    sn = inputs.anisotropic_orders(p["sigma_s"], 2, seed=203)
    print_case("pl_gg_diagonal", name=p["name"])
    nc = p["sigma_t"].shape[1]
    full = np.concatenate([p["sigma_s"][None], sn])
    gg = np.zeros((3, 2, 2, nc))
    for g in range(2):
        gg[:, g, g] = full[:, g]
    a = gpu_problem(api, ctx, p, "fp64")
    a.set_anisotropy(sn)
    phi_a, ia = a.source_iterate(tol=1e-12, max_iter=1000)
    b = gpu_problem(api, ctx, p, "fp64")
    b.set_anisotropy_gg(gg)
    phi_b, ib = b.source_iterate(tol=1e-12, max_iter=1000)
    assert ia["iters"] == ib["iters"]
    assert rel(phi_b.cpu().numpy(), phi_a.cpu().numpy()) <= 1e-13
    assert rel(b.moments().cpu().numpy(), a.moments().cpu().numpy()) <= 1e-12


def test_pl_gg_replace_clear_and_rejections(api, ctx):
    p = inputs.random_problem((4, 4, 3), 4, 2, seed=204)
    nc = p["sigma_t"].shape[1]
    sn = _multigroup_pl(p, 1, 205)
    print_case("pl_gg_rules", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp64")
    lib = api._lib.load()
    m = torch.tensor(sn, dtype=torch.float64, device="cuda")
    for order in (0, 4):
        assert lib.dgsn_problem_set_anisotropy_gg(prob._h, order, m.data_ptr(),
                                                  None) == api._lib.DGSN_EINVAL
    assert lib.dgsn_problem_set_anisotropy_gg(prob._h, 1, None, None) == api._lib.DGSN_EINVAL
    with pytest.raises(ValueError):
        prob.set_anisotropy_gg(sn[:1])
    # it replaces in-group orders set before
    prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], 2, seed=206))
    prob.set_anisotropy_gg(sn)
    phi, _ = prob.source_iterate(tol=1e-13, max_iter=1000)
    ref = _pl_gg_reference(p, sn)
    assert rel(phi.cpu().numpy(), ref["phi"]) <= 1e-10
    assert prob.moments().shape[0] == 3
    # exclusive with the separate calls while it is set
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.set_scattering(sn[0])
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], 1, seed=207))
    # clearing the orders keeps the order-0 group-to-group matrix
    prob.set_anisotropy(None)
    phi0, _ = prob.source_iterate(tol=1e-13, max_iter=1000)
    om, w = oracle.lq_n(p["order"])
    ref0 = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], np.zeros((2, nc)), p["q"],
                                 p["psi_inc"], tol=1e-14, max_iter=3000, sigma_gg=sn[0])
    assert rel(phi0.cpu().numpy(), ref0["phi"]) <= 1e-10


def test_pl_gg_many_groups(api, ctx):
    # more source groups than the 16 a thread stages in registers: the source
    # moments continue their sums over a second chunk of groups
    G = 18
    p = inputs.random_problem((3, 3, 2), 2, G, seed=208, length=(0.3, 0.3, 0.2))
    sn = _multigroup_pl(p, 1, 209, c=0.7)
    print_case("pl_gg_many_groups", name=p["name"], groups=G)
    for precision, bound in (("fp64", 1e-10), ("fp32", FP32_TOL)):
        prob = gpu_problem(api, ctx, p, precision)
        prob.set_anisotropy_gg(sn)
        tol = 1e-13 if precision == "fp64" else 1e-8
        phi, _ = prob.source_iterate(tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
        mom = prob.moments().double().cpu().numpy()
        prob.close()
        ref = _pl_gg_reference(p, sn)
        assert ref["converged"]
        for g in range(G):
            assert rel(phi.cpu().numpy()[g], ref["phi"][g]) <= bound, (precision, g)
        assert np.abs(mom - ref["mom"]).max() <= bound * np.abs(ref["phi"]).max()


def test_anisotropy_setters_fail_cleanly(api, ctx, monkeypatch):
    # an allocation failure part way through either setter (forced from the
    # host: allocations above DGSN_TEST_ALLOC_LIMIT are refused) leaves the
    # problem without anisotropic orders, so the next source iteration is the
    # isotropic one and reads no released buffer
    p = inputs.random_problem((5, 4, 4), 4, 2, seed=230, c_max=0.7)
    nc = p["sigma_t"].shape[1]
    print_case("pl_alloc_failure", name=p["name"])
    ref = gpu_problem(api, ctx, p, "fp32")
    phi_ref, _ = ref.source_iterate(tol=0.0, max_iter=5, allow_notconv=True)
    ref.close()
    mbytes = 3 * 2 * nc * 8 * 4          # one moment buffer at L = 1 (mom_oct is 8 of them)
    prob = gpu_problem(api, ctx, p, "fp32")
    prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], 1, seed=231))
    monkeypatch.setenv("DGSN_TEST_ALLOC_LIMIT", str(mbytes))
    with pytest.raises(api.DgsnError, match="ENOMEM"):
        prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], 2, seed=232))
    with pytest.raises(api.DgsnError, match="ENOMEM"):
        prob.set_anisotropy_gg(_multigroup_pl(p, 3, 233))
    monkeypatch.delenv("DGSN_TEST_ALLOC_LIMIT")
    assert prob.pl_order == 0
    lib = api._lib.load()
    out = torch.empty(1024, dtype=torch.float32, device="cuda")
    assert lib.dgsn_problem_get_moments(prob._h, out.data_ptr(), None) == api._lib.DGSN_EINVAL
    phi, _ = prob.source_iterate(tol=0.0, max_iter=5, allow_notconv=True)
    assert np.array_equal(phi.cpu().numpy(), phi_ref.cpu().numpy())
    # and the setters work again once allocations succeed
    prob.set_anisotropy_gg(_multigroup_pl(p, 1, 234))
    phi_gg, _ = prob.source_iterate(tol=1e-8, max_iter=1000, allow_notconv=True)
    assert rel(phi_gg.cpu().numpy(), _pl_gg_reference(p, _multigroup_pl(p, 1, 234))["phi"]) <= FP32_TOL


@pytest.mark.parametrize("gg", [False, True], ids=["in_group", "group_to_group"])
def test_pl_adjoint_schedules_and_tiles_bitwise(api, ctx, gg):
    # the anisotropic adjoint (reversed sweeps of the transposed cell systems
    # with the adjoint flux's moments) runs the same arithmetic under both
    # schedules; tile edges differ only by rounding
    p = inputs.random_problem((6, 5, 4), 4, 2, seed=240, c_max=0.7)
    print_case("pl_adjoint_schedules", name=p["name"], gg=gg)
    rng = np.random.default_rng(241)
    g = rng.uniform(0.0, 1.0, (2, p["sigma_t"].shape[1], 8))
    out = {}
    for sched in ("planes", "dataflow"):
        for b in (1, 2):
            prob = gpu_problem(api, ctx, p, "fp32", store_psi=True)
            if gg:
                prob.set_anisotropy_gg(_multigroup_pl(p, 1, 242, c=0.7))
            else:
                prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], 2, seed=243))
            prob.set_schedule(sched)
            prob.set_tile(b)
            prob.source_iterate(tol=0.0, max_iter=8, allow_notconv=True)
            gst, gq, _ = prob.adjoint(g, tol=0.0, max_iter=8, allow_notconv=True)
            out[(sched, b)] = (gst.cpu().numpy(), gq.cpu().numpy())
            prob.close()
    for b in (1, 2):
        assert np.array_equal(out[("planes", b)][0], out[("dataflow", b)][0])
        assert np.array_equal(out[("planes", b)][1], out[("dataflow", b)][1])
    assert rel(out[("planes", 2)][1], out[("planes", 1)][1]) <= 1e-4


@pytest.mark.parametrize("precision,L", [("fp64", 1), ("fp64", 2), ("fp32", 2)])
def test_pl_gg_adjoint_matches_oracle(api, ctx, precision, L):
    p = inputs.random_problem((5, 4, 4), 4, 3, seed=210 + L, length=(0.5, 0.4, 0.4))
    sn = _multigroup_pl(p, L, 215 + L, c=0.7)
    print_case("pl_gg_adjoint", name=p["name"], precision=precision, L=L)
    prob = gpu_problem(api, ctx, p, precision, store_psi=True)
    prob.set_anisotropy_gg(sn)
    tol = 1e-13 if precision == "fp64" else 1e-7
    prob.source_iterate(tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    rng = np.random.default_rng(220 + L)
    g = rng.uniform(0.0, 1.0, (3, p["sigma_t"].shape[1], 8))
    gst, gq, info = prob.adjoint(g, tol=tol, max_iter=1000, allow_notconv=precision == "fp32")
    om, w = oracle.lq_n(p["order"])
    r = _pl_gg_reference(p, sn, store_psi=True)
    zero = np.zeros_like(p["sigma_t"])
    a = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], zero, r["psi"], r["phi"], g,
                       tol=1e-15, sigma_sn=sn, pl_gg=True)
    bound = 1e-9 if precision == "fp64" else 1e-4
    assert rel(gst.cpu().numpy(), a["grad_sigma_t"]) <= bound
    assert rel(gq.cpu().numpy(), a["grad_q"]) <= bound
    # the transpose matters: the adjoint of the untransposed coupling differs
    snt = np.ascontiguousarray(np.swapaxes(sn, 1, 2))
    wrong = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], zero, r["psi"], r["phi"], g,
                           tol=1e-15, sigma_sn=snt, pl_gg=True)
    assert rel(wrong["grad_q"], a["grad_q"]) > 100 * bound


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("solver", ["ge", "ge_dense"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_adjoint_matches_oracle(api, ctx, precision, tol, solver, tile):
    p = inputs.adjoint_box(n=7, groups=2, seed=4, box=(2, 5))
    print_case("adjoint", name=p["name"], precision=precision, solver=solver, tile=tile)
    prob = gpu_problem(api, ctx, p, precision, solver=solver, store_psi=True)
    prob.set_tile(tile)
    si_tol = 1e-13 if precision == "fp64" else 1e-7
    phi, info = prob.source_iterate(tol=si_tol, max_iter=1000, allow_notconv=True)
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    g = np.zeros((p["groups"], 343, 8))
    g[:, p["box_mask"], :] = ((p["sigma_t"] - p["sigma_s"])[:, p["box_mask"]] * V / 8)[..., None]
    dt = torch.float64 if precision == "fp64" else torch.float32
    gst, gq, ainfo = prob.adjoint(torch.tensor(g, dtype=dt, device="cuda"), tol=si_tol,
                                  max_iter=1000, allow_notconv=True)
    om, w = oracle.lq_n(p["order"])
    ref = oracle.source_iterate(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-14, max_iter=2000, store_psi=True)
    a = oracle.adjoint(mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], ref["psi"], ref["phi"], g,
                       tol=1e-14)
    assert rel(gst.cpu().numpy(), a["grad_sigma_t"]) <= tol
    assert rel(gq.cpu().numpy(), a["grad_q"]) <= tol


# ---------------------------------------------------------------------------
# ANN
# ---------------------------------------------------------------------------

def _random_net(seed, nh=64):
    rng = np.random.default_rng(seed)
    return dict(W1=(rng.normal(size=(nh, 24)) / 5).astype(np.float32),
                b1=(rng.normal(size=nh) / 5).astype(np.float32),
                W2=(rng.normal(size=(8, nh)) / 8).astype(np.float32),
                b2=(rng.normal(size=8) / 5).astype(np.float32))


def _write_net(tmp_path, net, name):
    from paper_1906_04017_amd import ann_format
    path = tmp_path / name
    ann_format.write(path, net["W1"], net["b1"], net["W2"], net["b2"])
    return path


@pytest.mark.parametrize("nh", [64, 40, 8])
def test_ann_infer_within_bf16_bound(api, ctx, tmp_path, nh):
    print_case("ann_infer", nh=nh)
    net = _random_net(300 + nh, nh)
    ann = api.Ann(ctx, _write_net(tmp_path, net, f"r{nh}.dgsnann"))
    rng = np.random.default_rng(7)
    n = 1000 + 37
    x = rng.uniform(-1, 1, size=(n, 24)).astype(np.float32)
    y = ann.infer(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    W1, b1, W2, b2 = (net[k].astype(np.float64) for k in ("W1", "b1", "W2", "b2"))
    xd = x.astype(np.float64)
    ref = np.stack([oracle.ann_forward(net, xi) for xi in xd])
    hid = np.maximum(xd @ W1.T + b1, 0)
    u = 3 * 2.0 ** -8
    dh = u * (np.abs(xd) @ np.abs(W1).T + np.abs(b1))
    bound = u * (np.abs(hid) @ np.abs(W2).T + np.abs(b2)) + (dh @ np.abs(W2).T)
    assert np.all(np.abs(y - ref) <= bound + 1e-6)


def _identity_net(select):
    W1 = np.zeros((48, 24))
    for j in range(24):
        W1[2 * j, j] = 1.0
        W1[2 * j + 1, j] = -1.0
    W2 = np.zeros((8, 48))
    for t, j in enumerate(select):
        W2[t, 2 * j] = 1.0
        W2[t, 2 * j + 1] = -1.0
    return dict(W1=W1.astype(np.float32), b1=np.zeros(48, np.float32),
                W2=W2.astype(np.float32), b2=np.zeros(8, np.float32))


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_ann_sweep_source_passthrough_net(api, ctx, tmp_path, tile):
    # psi = h S exactly (network y[n'] = x[16 + n']): checks features,
    # reflection, normalisation and rescaling of the ANN sweep kernel; the
    # only error is BF16 rounding of the normalised input and hidden value
    net = _identity_net([16 + n for n in range(8)])
    ann = api.Ann(ctx, _write_net(tmp_path, net, "src_pass.dgsnann"))
    p = inputs.random_problem((7, 5, 6), 6, 2, seed=31, length=(0.7, 0.5, 0.6))
    print_case("ann_sweep_source_passthrough", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    prob.set_tile(tile)
    S = nodal_source(p, seed=13)
    phi = prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(6)
    ref = oracle.ann_sweep(net, mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= 2 * 2.0 ** -8


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_ann_sweep_inflow_passthrough_net(api, ctx, tmp_path, tile):
    # psi[n] = x-face inflow at the partner node: values are copied cell to
    # cell along x, so the fronts and their boundary values are exercised;
    # each hop re-rounds to BF16 at most twice
    sel = [4 + (((n >> 1) & 1) + 2 * ((n >> 2) & 1)) for n in range(8)]
    net = _identity_net(sel)
    ann = api.Ann(ctx, _write_net(tmp_path, net, "inflow_pass.dgsnann"))
    p = inputs.random_problem((6, 4, 3), 4, 1, seed=33)
    p["psi_inc"] = np.array([0.8, 0.3, 0.0, 0.0, 0.0, 0.0])
    p["q"][:] = 0.0
    print_case("ann_sweep_inflow_passthrough", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    prob.set_tile(tile)
    S = nodal_source(p)
    phi = prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(4)
    ref = oracle.ann_sweep(net, mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= 2 * 6 * 2.0 ** -8


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_ann_dataflow_matches_planes_bitwise(api, ctx, tmp_path, tile):
    # the matrix-core network under the one-launch dataflow schedule runs the
    # same per-cell arithmetic as under the hyperplane launches
    net = _random_net(91)
    ann = api.Ann(ctx, _write_net(tmp_path, net, "flow_ann.dgsnann"))
    p = inputs.random_problem((9, 7, 8), 8, 3, seed=92, length=(0.9, 0.7, 0.8))
    print_case("ann_dataflow", name=p["name"], tile=tile)
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    prob.set_tile(tile)
    S = torch.tensor(nodal_source(p, seed=93), dtype=torch.float32, device="cuda")
    ref = prob.sweep(S).clone()
    prob.set_schedule("dataflow")
    for _ in range(3):
        got = prob.sweep(S)
        prob.check()
        assert torch.equal(got, ref)


# ---------------------------------------------------------------------------
# paper-form per-octant network (26 inputs, tanh, ELU; vector ALUs)
# ---------------------------------------------------------------------------

def _random_pann(seed, nh=8):
    rng = np.random.default_rng(seed)
    imin, imax = np.zeros(26), np.ones(26)
    imin[12:14] = -1.0
    imax[22] = 10.0
    imin[23:26] = 0.1
    return dict(W1=(rng.normal(size=(8, nh, 26)) / 5), b1=(rng.normal(size=(8, nh)) / 5),
                W2=(rng.normal(size=(8, 8, nh)) / 8), b2=(np.abs(rng.normal(size=(8, 8))) / 5),
                imin=imin, imax=imax)


def _write_pann(tmp_path, net, name):
    """Writes the artifact and returns (path, the stored network as the oracle
    reads it: float32 parameters)."""
    from oracle import ann_paper_train
    from paper_1906_04017_amd import ann_format
    path = tmp_path / name
    ann_format.write_paper(path, net["W1"], net["b1"], net["W2"], net["b2"], net["imin"],
                           net["imax"])
    # the oracle reads the artifact with its own reader
    return path, ann_paper_train.read_artifact(path)


def _pann_bound(net, o, I):
    """Bound on |FP32 device - FP64| for one sample of octant o's network: the
    scaling is folded into the first layer (one rounding per weight), the
    sums are FP32 (at most 30 roundings of the largest partial sum), tanh and
    exp come from the hardware exp2 and reciprocal (a few 1e-8 absolute)."""
    u = 2.0 ** -24
    W1, b1 = net["W1"][o].astype(np.float64), net["b1"][o].astype(np.float64)
    W2, b2 = net["W2"][o].astype(np.float64), net["b2"][o].astype(np.float64)
    c = net["alpha"] * 0.5 * (net["imin"] + net["imax"])
    r = np.abs(net["imax"] - net["imin"])
    Wf = W1 / r[None, :]
    bf = b1 - Wf @ c
    dz = 30 * u * (np.abs(Wf) @ np.abs(I) + np.abs(bf) + np.abs(Wf) @ np.abs(c))
    h = np.tanh(Wf @ I + bf)
    dh = dz + 2e-7
    do = np.abs(W2) @ dh + 12 * u * (np.abs(W2) @ np.abs(h) + np.abs(b2))
    beta = net["beta_scale"] * I[:12].max()
    return max(1.0, beta) * do + 4e-7 * beta


@pytest.mark.parametrize("nh", [8, 5])
def test_pann_infer_octant_within_fp32_bound(api, ctx, tmp_path, nh):
    print_case("pann_infer", nh=nh)
    path, net = _write_pann(tmp_path, _random_pann(400 + nh, nh), f"p{nh}.dgsnann")
    ann = api.Ann(ctx, path)
    assert ann.info() == (2, 26, nh, 8)
    rng = np.random.default_rng(9)
    n = 700 + 13
    x = rng.uniform(-0.2, 1.2, size=(n, 26))
    x[:, 22] *= 10.0
    x = x.astype(np.float32)
    xd = x.astype(np.float64)
    for o in range(8):
        y = ann.infer_octant(o, torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
        for i in range(0, n, 7):
            ref = oracle.pann_forward(net, o, xd[i])
            assert np.all(np.abs(y[i] - ref) <= 2 * _pann_bound(net, o, xd[i]) + 1e-7), (o, i)
    with pytest.raises(Exception):
        ann.infer(torch.zeros((4, 24), device="cuda"))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_set_materials_rejects_invalid_values(api, ctx, precision):
    p = inputs.random_problem((4, 3, 3), 4, 2, seed=236, c_max=0.5)
    print_case("invalid_materials", name=p["name"], precision=precision)
    prob = gpu_problem(api, ctx, p, precision)
    st, ss, q = p["sigma_t"].copy(), p["sigma_s"].copy(), p["q"].copy()
    cases = [("sigma_t", dict(st=np.nan)), ("sigma_t", dict(st=-0.5)), ("sigma_t", dict(st=np.inf)),
             ("sigma_s", dict(ss=-1e-3)), ("sigma_s", dict(ss=np.nan)), ("q", dict(q=-np.inf)),
             ("sigma_s exceeds", dict(ss=st[0, 3] * 1.01))]
    for name, bad in cases:
        a, b, c = st.copy(), ss.copy(), q.copy()
        if "st" in bad: a[1, 7] = bad["st"]
        if "ss" in bad: b[0, 3] = bad["ss"]
        if "q" in bad: c[1, 0] = bad["q"]
        with pytest.raises(api.DgsnError, match=f"EINVAL.*{name}"):
            prob.set_materials(a, b, c)
    # zero cross sections and a negative (finite) source are valid
    z = np.zeros_like(st)
    prob.set_materials(z, z, -q)
    prob.set_materials(st, ss, q)
    phi, info = prob.source_iterate(tol=1e-6, max_iter=500, allow_notconv=True)
    om, w = oracle.lq_n(4)
    ref = oracle.source_iterate(mesh_of(p), om, w, st, ss, q, p["psi_inc"], tol=1e-12,
                                max_iter=3000)
    assert rel(phi.cpu().numpy(), ref["phi"]) <= 1e-4


def test_set_ann_failure_leaves_no_network(api, ctx, tmp_path, monkeypatch):
    # the per-problem image of a paper-form network cannot be allocated
    # (forced from the host): the problem is left with no network, so a
    # sweep reports the missing network instead of reading a released image
    path, _ = _write_pann(tmp_path, _random_pann(410), "pf.dgsnann")
    ann = api.Ann(ctx, path)
    p = inputs.random_problem((4, 4, 3), 4, 1, seed=235)
    print_case("set_ann_failure", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    src = torch.ones((1, p["sigma_t"].shape[1], 8), dtype=torch.float32, device="cuda")
    good = prob.sweep(src).cpu().numpy()
    monkeypatch.setenv("DGSN_TEST_ALLOC_LIMIT", "64")
    with pytest.raises(api.DgsnError, match="ENOMEM"):
        prob.set_ann(ann)
    monkeypatch.delenv("DGSN_TEST_ALLOC_LIMIT")
    with pytest.raises(api.DgsnError, match="EINVAL"):
        prob.sweep(src)
    prob.set_ann(ann)
    assert np.array_equal(prob.sweep(src).cpu().numpy(), good)


PANN_CASES = [((5, 4, 6), (0.5, 0.4, 0.6), 4, 2), ((7, 5, 6), (0.7, 0.5, 0.6), 6, 1),
              ((3, 8, 2), (0.3, 0.8, 0.2), 8, 3)]


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("case", PANN_CASES, ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in PANN_CASES])
def test_pann_sweep_matches_oracle(api, ctx, tmp_path, case, tile):
    n, L, order, G = case
    print_case("pann_sweep", n=n, order=order, G=G, tile=tile)
    path, net = _write_pann(tmp_path, _random_pann(500), "ps.dgsnann")
    ann = api.Ann(ctx, path)
    p = inputs.random_problem(n, order, G, seed=61 + tile, length=L)
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    prob.set_tile(tile)
    S = torch.tensor(nodal_source(p, seed=17), dtype=torch.float32, device="cuda")
    phi = prob.sweep(S).clone()
    om, w = oracle.lq_n(order)
    ref = oracle.pann_sweep(net, mesh_of(p), om, w, p["sigma_t"], S.cpu().numpy(), p["psi_inc"])
    assert rel(phi.cpu().numpy(), ref) <= 2e-5
    # the dataflow schedule runs the same arithmetic
    prob.set_schedule("dataflow")
    for _ in range(2):
        got = prob.sweep(S)
        prob.check()
        assert torch.equal(got, phi)


def test_pann_source_iteration_matches_oracle(api, ctx, tmp_path):
    path, net = _write_pann(tmp_path, _random_pann(501), "psi.dgsnann")
    ann = api.Ann(ctx, path)
    p = inputs.random_problem((6, 5, 4), 4, 2, seed=71, c_max=0.5, length=(0.6, 0.5, 0.4))
    print_case("pann_si", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    phi, info = prob.source_iterate(tol=1e-6, max_iter=200)
    om, w = oracle.lq_n(4)
    ref = oracle.pann_source_iterate(net, mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                     p["psi_inc"], tol=1e-10, max_iter=500)
    assert rel(phi.cpu().numpy(), ref["phi"]) <= 5e-5


def test_pann_rejects_fp64_and_adjoint(api, ctx, tmp_path):
    path, _ = _write_pann(tmp_path, _random_pann(502), "pe.dgsnann")
    ann = api.Ann(ctx, path)
    p = inputs.random_problem((3, 3, 3), 2, 1, seed=72)
    prob64 = gpu_problem(api, ctx, p, "fp64")
    with pytest.raises(Exception):
        prob64.set_ann(ann)
    probs = gpu_problem(api, ctx, p, "fp32", solver="ann", store_psi=True)
    probs.set_ann(ann)
    with pytest.raises(Exception):
        probs.sweep(torch.zeros((1, 27, 8), device="cuda"))


# ---------------------------------------------------------------------------
# dataflow schedule (one launch per sweep, device counters between steps)
# ---------------------------------------------------------------------------

FLOW_CASES = RAGGED + [((24, 20, 18), (1.2, 1.0, 0.9), 8, 3)]


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", FLOW_CASES, ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in FLOW_CASES])
def test_dataflow_matches_planes_bitwise(api, ctx, precision, case, tile):
    # same arithmetic in the same order: any stale front read across the
    # device's caches would show up as a difference
    n, L, order, G = case
    print_case("dataflow", n=n, order=order, G=G, precision=precision, tile=tile)
    p = inputs.random_problem(n, order, G, seed=(hash(case) + 1) % 1000, length=L)
    prob = gpu_problem(api, ctx, p, precision)
    prob.set_tile(tile)
    dt = torch.float64 if precision == "fp64" else torch.float32
    S = torch.tensor(nodal_source(p, seed=8), dtype=dt, device="cuda")
    ref = prob.sweep(S).clone()
    prob.set_schedule("dataflow")
    assert prob.schedule() == "dataflow"
    for _ in range(3):
        got = prob.sweep(S)
        prob.check()
        assert torch.equal(got, ref)
    om, w = oracle.lq_n(order)
    want = oracle.sweep(mesh_of(p), om, w, p["sigma_t"], S.cpu().numpy(), p["psi_inc"])
    assert rel(got.cpu().numpy(), want) <= (FP64_SWEEP_TOL if precision == "fp64" else FP32_TOL)


def test_dataflow_source_iteration_and_adjoint(api, ctx):
    p = inputs.adjoint_box(n=7, groups=2, seed=4, box=(2, 5))
    print_case("dataflow_si_adjoint", name=p["name"])
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    g = np.zeros((p["groups"], 343, 8))
    g[:, p["box_mask"], :] = ((p["sigma_t"] - p["sigma_s"])[:, p["box_mask"]] * V / 8)[..., None]
    out = {}
    for sched in ("planes", "dataflow"):
        prob = gpu_problem(api, ctx, p, "fp64", store_psi=True)
        prob.set_tile(2)
        prob.set_schedule(sched)
        phi, info = prob.source_iterate(tol=1e-13, max_iter=1000)
        gst, gq, _ = prob.adjoint(torch.tensor(g, device="cuda"), tol=1e-13, max_iter=1000)
        out[sched] = (phi.cpu(), gst.cpu(), gq.cpu(), info["iters"])
    a, b = out["planes"], out["dataflow"]
    assert a[3] == b[3]
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_dataflow_expired_wait_is_reported(api, ctx):
    # a column of 64 cells: the unit of the last step waits for 63 sequential
    # solves, far beyond a poll limit of 1; the launch must still complete,
    # the host must report the expired wait, and the next sweep (default
    # limit) must be exact again
    p = inputs.random_problem((1, 1, 64), 2, 1, seed=5, length=(0.1, 0.1, 6.4))
    print_case("dataflow_expired_wait", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32")
    prob.set_tile(1)
    S = torch.tensor(nodal_source(p, seed=3), dtype=torch.float32, device="cuda")
    ref = prob.sweep(S).clone()
    prob.set_schedule("dataflow", poll_limit=1)
    prob.sweep(S)
    with pytest.raises(api.DgsnError, match="DGSN_ETIMEOUT.*dataflow"):
        prob.check()
    prob.check()   # the condition was cleared
    prob.set_schedule("dataflow")
    got = prob.sweep(S)
    prob.check()
    assert torch.equal(got, ref)


# ---------------------------------------------------------------------------
# poisoned fronts (debug mode): every front slot a sweep reads was written
# earlier in the same sweep
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", RAGGED[:3], ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in RAGGED[:3]])
def test_poisoned_fronts_leave_sweeps_unchanged(api, ctx, precision, case):
    n, L, order, G = case
    p = inputs.random_problem(n, order, G, seed=170, length=L, c_max=0.5)
    print_case("poison_fronts", name=p["name"], precision=precision)
    dt = torch.float32 if precision == "fp32" else torch.float64
    S = torch.tensor(nodal_source(p, seed=171), dtype=dt, device="cuda")
    for solver in (("ge", "ge_dense") if precision == "fp32" else ("ge",)):
        prob = gpu_problem(api, ctx, p, precision, solver=solver)
        for sched in ("planes", "dataflow"):
            prob.set_schedule(sched)
            for b in (1, 2, 3):
                prob.set_tile(b)
                prob.set_debug(poison_fronts=False)
                ref = prob.sweep(S).clone()
                prob.set_debug(poison_fronts=True)
                got = prob.sweep(S)
                prob.check()
                assert torch.equal(got, ref), (solver, sched, b)
                assert torch.isfinite(got).all()
        # a poisoned source iteration converges to the same iterate
        prob.set_debug(poison_fronts=False)
        a, ia = prob.source_iterate(tol=1e-7, max_iter=300, allow_notconv=True)
        prob.set_debug(poison_fronts=True)
        b2, ib = prob.source_iterate(tol=1e-7, max_iter=300, allow_notconv=True)
        assert torch.equal(a, b2) and ia["iters"] == ib["iters"]
        prob.close()
    with pytest.raises(api.DgsnError, match="EINVAL"):
        _lib_set_debug(api, p, ctx, 2)


def _lib_set_debug(api, p, ctx, flags):
    from paper_1906_04017_amd import _lib
    prob = gpu_problem(api, ctx, p, "fp32")
    try:
        _lib.check(_lib.load().dgsn_problem_set_debug(prob._h, flags))
    finally:
        prob.close()


# ---------------------------------------------------------------------------
# autotuner and batched execution
# ---------------------------------------------------------------------------

def test_problem_autotune_keeps_results(api, ctx):
    p = inputs.random_problem((10, 9, 8), 6, 3, seed=51)
    print_case("autotune", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32")
    tile, sched, times = prob.autotune()
    assert tile in (1, 2, 3) and sched in ("planes", "dataflow") and len(times) == 6
    assert min(times.values()) > 0 and times[(sched, tile)] == min(times.values())
    assert prob.schedule() == sched
    assert prob.tile() == tile
    S = nodal_source(p, seed=5)
    phi = prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(6)
    ref = oracle.sweep(mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    assert rel(phi, ref) <= FP32_TOL


def test_autotune_cache_reuses_choices(api, ctx, tmp_path):
    # a second problem of the same shape takes the first one's choice and
    # times without timing again (the times come back identical); the cache
    # survives a save, clear and load; another shape is timed anew
    api.autotune_cache_clear()
    p = inputs.random_problem((9, 8, 7), 8, 2, seed=53)
    print_case("autotune_cache", name=p["name"])
    a = gpu_problem(api, ctx, p, "fp32")
    first = a.autotune()
    assert api.autotune_cache_size() == 1
    q = dict(p, sigma_t=p["sigma_t"] * 1.5)
    b = gpu_problem(api, ctx, q, "fp32")
    assert b.autotune() == first
    assert b.schedule() == first[1] and b.tile() == first[0]
    path = tmp_path / "tune.json"
    api.autotune_cache_save(path)
    api.autotune_cache_clear()
    api.autotune_cache_load(path)
    c = gpu_problem(api, ctx, p, "fp32")
    assert c.autotune() == first
    # the cached choice sweeps correctly (a dataflow choice builds its tables)
    S = nodal_source(q, seed=6)
    phi = b.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")).cpu().numpy()
    om, w = oracle.lq_n(8)
    assert rel(phi, oracle.sweep(mesh_of(q), om, w, q["sigma_t"], S, q["psi_inc"])) <= FP32_TOL
    d = gpu_problem(api, ctx, inputs.random_problem((9, 8, 6), 8, 2, seed=54), "fp32")
    d.autotune()
    assert api.autotune_cache_size() == 2
    for prob in (a, b, c, d):
        prob.close()


BATCH = [((5, 4, 3), 4, 2, "ge"), ((9, 9, 9), 8, 3, "ge"), ((3, 7, 2), 12, 1, "ge"),
         ((6, 5, 4), 6, 2, "ann"), ((1, 1, 1), 2, 1, "ge"), ((8, 6, 7), 4, 4, "ann"),
         ((12, 10, 11), 8, 2, "ge"), ((7, 6, 5), 6, 3, "pann"), ((9, 4, 6), 4, 2, "pann")]


@pytest.mark.parametrize("schedule", ["planes", "dataflow"])
@pytest.mark.parametrize("tiles", ["default", "ones", "autotune"])
def test_batch_matches_single_problem_sweeps(api, ctx, tmp_path, tiles, schedule):
    print_case("batch", tiles=tiles, schedule=schedule, problems=len(BATCH))
    net = _random_net(77)
    ann = api.Ann(ctx, _write_net(tmp_path, net, "batch.dgsnann"))
    pann = api.Ann(ctx, _write_pann(tmp_path, _random_pann(78), "batch_p.dgsnann")[0])
    probs, srcs, phis, ps = [], [], [], []
    for k, (n, order, G, solver) in enumerate(BATCH):
        p = inputs.random_problem(n, order, G, seed=600 + k,
                                  length=tuple(0.1 * v + 0.3 for v in n))
        prob = gpu_problem(api, ctx, p, "fp32", solver="ge" if solver == "ge" else "ann")
        if solver == "ann":
            prob.set_ann(ann)
        if solver == "pann":
            prob.set_ann(pann)
        S = torch.tensor(nodal_source(p, seed=700 + k), dtype=torch.float32, device="cuda")
        probs.append(prob)
        srcs.append(S)
        phis.append(torch.full_like(S, float("nan")))
        ps.append(p)
    batch = api.Batch(ctx, probs)
    for k in range(len(probs)):
        batch.set_io(k, srcs[k], phis[k])
    batch.set_schedule(schedule)
    if tiles == "ones":
        batch.set_tiles([1] * len(probs))
    elif tiles == "autotune":
        assert batch.autotune() > 0
        assert batch.schedule() in ("planes", "dataflow")
    for _ in range(2):   # a graph replay must give the same results
        for ph in phis:
            ph.fill_(float("nan"))
        batch.run()
        torch.cuda.synchronize()
    lat = batch.latencies_us()
    assert np.all(lat > 0)
    for k, (n, order, G, solver) in enumerate(BATCH):
        got = phis[k].cpu().numpy()
        if solver == "ge":
            om, w = oracle.lq_n(order)
            ref = oracle.sweep(mesh_of(ps[k]), om, w, ps[k]["sigma_t"], srcs[k].cpu().numpy(),
                               ps[k]["psi_inc"])
            assert rel(got, ref) <= FP32_TOL, (k, rel(got, ref))
        else:
            # same device arithmetic as the single-problem ANN sweep
            ref = probs[k].sweep(srcs[k]).cpu().numpy()
            assert np.array_equal(got, ref), k
    batch.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_transport_solve_autograd(api, ctx, precision, tol):
    # J = sum_box (sigma_t - sigma_s) int phi through torch autograd: the
    # direct term by torch, the solve term by the adjoint sweep; against the
    # oracle's adjoint plus the same direct term
    p = inputs.adjoint_box(n=6, groups=2, seed=9, box=(1, 4))
    print_case("autograd", name=p["name"], precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision=precision,
                       store_psi=True)
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    box = torch.tensor(p["box_mask"], device="cuda")
    st = torch.tensor(p["sigma_t"], dtype=dt, device="cuda", requires_grad=True)
    q = torch.tensor(p["q"], dtype=dt, device="cuda", requires_grad=True)
    ss = torch.tensor(p["sigma_s"], dtype=dt, device="cuda")
    si_tol = 1e-13 if precision == "fp64" else 1e-7
    phi = api.TransportSolve.apply(prob, st, q, ss, si_tol, 2000)
    J = (((st - ss) * box)[..., None] * phi).sum() * (V / 8)
    J.backward()
    om_o, w_o = oracle.lq_n(p["order"])
    mesh = mesh_of(p)
    ref = oracle.source_iterate(mesh, om_o, w_o, p["sigma_t"], p["sigma_s"], p["q"],
                                p["psi_inc"], tol=1e-14, max_iter=3000, store_psi=True)
    g = np.zeros((p["groups"], 216, 8))
    g[:, p["box_mask"], :] = ((p["sigma_t"] - p["sigma_s"])[:, p["box_mask"]] * V / 8)[..., None]
    a = oracle.adjoint(mesh, om_o, w_o, p["sigma_t"], p["sigma_s"], ref["psi"], ref["phi"], g,
                       tol=1e-14)
    direct = p["box_mask"][None, :] * ref["phi"].sum(-1) * (V / 8)
    assert rel(st.grad.cpu().numpy(), a["grad_sigma_t"] + direct) <= tol
    assert rel(q.grad.cpu().numpy(), a["grad_q"]) <= tol


# ---------------------------------------------------------------------------
# split-BF16 evaluation of the matrix-core network
# ---------------------------------------------------------------------------

def _bf16_exact(a):
    """a rounded to the nearest BF16 value (ties to even), as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("nh", [64, 40])
def test_ann_infer_split_bf16_within_bound(api, ctx, tmp_path, nh):
    # weights held exactly in BF16 (as the trainer writes them): the split
    # mode carries every feature and hidden activation as hi + lo to 2^-18
    # relative (hi = bf16(v) to 2^-9, lo = bf16(v - hi) to 2^-9 of the rest),
    # the bias likewise, products are exact in FP32 and the K <= 64 FP32 sums
    # add at most 64 * 2^-24 relative to the absolute sums: 4 * 2^-18 covers
    # both for each layer
    print_case("ann_infer_split", nh=nh)
    net = {k: _bf16_exact(v) for k, v in _random_net(310 + nh, nh).items()}
    ann = api.Ann(ctx, _write_net(tmp_path, net, f"s{nh}.dgsnann"))
    ann.set_mode("bf16x2")
    rng = np.random.default_rng(8)
    n = 1000 + 41
    x = rng.uniform(-1, 1, size=(n, 24)).astype(np.float32)
    y = ann.infer(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    W1, b1, W2, b2 = (net[k].astype(np.float64) for k in ("W1", "b1", "W2", "b2"))
    xd = x.astype(np.float64)
    ref = np.stack([oracle.ann_forward(net, xi) for xi in xd])
    hid = np.maximum(xd @ W1.T + b1, 0)
    u = 4 * 2.0 ** -18
    dh = u * (np.abs(xd) @ np.abs(W1).T + np.abs(b1))
    bound = u * (np.abs(hid) @ np.abs(W2).T + np.abs(b2)) + (dh @ np.abs(W2).T)
    err = np.abs(y - ref)
    assert np.all(err <= bound + 2.0 ** -22 * np.abs(ref))
    # and well below the BF16 mode's error on the same inputs
    ann.set_mode("bf16")
    y16 = ann.infer(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    assert err.max() < np.abs(y16 - ref).max() / 50
    ann.close()


def test_ann_split_mode_rules(api, ctx, tmp_path):
    print_case("ann_split_rules")
    pann = api.Ann(ctx, _write_pann(tmp_path, _random_pann(91), "rules_p.dgsnann")[0])
    with pytest.raises(api.DgsnError, match="EINVAL"):
        pann.set_mode("bf16x2")
    pann.set_mode("bf16")
    ann = api.Ann(ctx, _write_net(tmp_path, _random_net(92), "rules.dgsnann"))
    ann.set_mode("bf16x2")
    p = inputs.random_problem((4, 3, 3), 4, 1, seed=93)
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    S = torch.tensor(nodal_source(p), dtype=torch.float32, device="cuda")
    batch = api.Batch(ctx, [prob])
    batch.set_io(0, S, torch.empty_like(S))
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        batch.run()
    ann.set_mode("bf16")
    batch.run()
    torch.cuda.synchronize()
    batch.close()
    prob.close()


@pytest.mark.parametrize("schedule", ["planes", "dataflow"])
@pytest.mark.parametrize("tile", [1, 2, 3])
def test_ann_split_sweep_matches_fp64_forward(api, ctx, tmp_path, tile, schedule):
    # a BF16-exact network in a whole sweep (ragged mesh, S6, 2 groups)
    # against the oracle's FP64 forward of the same artifact in the same
    # sweep: the per-cell network error (about 2^-16 of its output) carried
    # downstream; the BF16 mode on the same sweep is far off in comparison
    net = {k: _bf16_exact(v) for k, v in _random_net(95, 64).items()}
    net["W2"] = _bf16_exact(net["W2"] * 0.25)   # a contracting network
    ann = api.Ann(ctx, _write_net(tmp_path, net, "split_sweep.dgsnann"))
    ann.set_mode("bf16x2")
    p = inputs.random_problem((7, 5, 6), 6, 2, seed=96, length=(0.7, 0.5, 0.6))
    print_case("ann_split_sweep", name=p["name"], tile=tile, schedule=schedule)
    prob = gpu_problem(api, ctx, p, "fp32", solver="ann")
    prob.set_ann(ann)
    prob.set_tile(tile)
    prob.set_schedule(schedule)
    S = nodal_source(p, seed=97)
    St = torch.tensor(S, dtype=torch.float32, device="cuda")
    phi = prob.sweep(St).cpu().numpy()
    om, w = oracle.lq_n(6)
    ref = oracle.ann_sweep(net, mesh_of(p), om, w, p["sigma_t"], S, p["psi_inc"])
    e_split = rel(phi, ref)
    assert e_split <= 32 * 2.0 ** -18, e_split
    ann.set_mode("bf16")
    e16 = rel(prob.sweep(St).cpu().numpy(), ref)
    assert e_split < e16 / 20, (e_split, e16)
    prob.close()
    ann.close()

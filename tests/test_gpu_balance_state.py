"""GPU checks of the particle-balance tally and of the problem state rules.

The balance tally (FP64 sums of the boundary outflow and inflow, absorption
and source of a sweep; the weak form below Eq. (T9) tested with 1) is
compared with the oracle's term-by-term balance of the same sweep computed
from its stored angular flux.  The state checks cover what a caller must not
be able to get wrong silently: a NaN flux reported as converged, an expired
dataflow wait, a batch graph that still holds a changed inflow or network, an
adjoint run against a stale angular flux, and an autograd backward after the
problem changed.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1906_04017_amd import inputs

pytestmark = pytest.mark.gpu

_DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1906_04017_amd", "data")
ARTIFACTS = {"paper": os.path.join(_DATA, "ann_paper_tanh8.dgsnann"),
             "mfma": os.path.join(_DATA, "ann_s8_relu64.dgsnann")}


@pytest.fixture(scope="module")
def api():
    from paper_1906_04017_amd import api as _api
    return _api


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


def print_case(case, **kw):
    print(f"[case] {case} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def gpu_problem(api, ctx, p, precision, solver="ge", store_psi=False):
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision=precision,
                       solver=solver, store_psi=store_psi)
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    return prob


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ---------------------------------------------------------------------------
# particle-balance tally
# ---------------------------------------------------------------------------

BAL_CASES = [((5, 3, 4), (1.0, 0.6, 0.8), 4, 2), ((7, 2, 9), (0.7, 0.2, 1.8), 8, 1),
             ((1, 1, 1), (0.3, 0.3, 0.3), 2, 1)]


@pytest.mark.parametrize("schedule", ["planes", "dataflow"])
@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
@pytest.mark.parametrize("case", BAL_CASES, ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in BAL_CASES])
def test_balance_tally_matches_oracle(api, ctx, case, precision, tol, tile, schedule):
    n, L, order, G = case
    p = inputs.random_problem(n, order, G, seed=801, length=L)
    print_case("balance", name=p["name"], precision=precision, tile=tile, schedule=schedule)
    prob = gpu_problem(api, ctx, p, precision)
    prob.set_tile(tile)
    prob.set_schedule(schedule)
    prob.set_balance(True)
    S = np.repeat(p["q"][..., None], 8, axis=-1) + \
        inputs.random_nodal(p["sigma_t"].shape[1], G, 802, -0.2, 0.5)
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob.sweep(torch.tensor(S, dtype=dt, device="cuda"))
    got = prob.balance()
    om, w = oracle.lq_n(order)
    mesh = (*p["n"], *p["length"])
    _, psi = oracle.sweep(mesh, om, w, p["sigma_t"], S, p["psi_inc"], store_psi=True)
    ref = oracle.sweep_balance(mesh, om, w, p["sigma_t"], S, p["psi_inc"], psi)
    scale = ref["inflow"] + abs(ref["source"]) + ref["absorption"]
    for key in ("outflow", "inflow", "absorption", "source"):
        assert abs(got[key] - ref[key]) <= tol * scale, (key, got[key], ref[key])
    assert abs(got["balance"]) <= tol * scale
    # the tally does not change the sweep's results
    prob.set_balance(False)
    phi0 = prob.sweep(torch.tensor(S, dtype=dt, device="cuda")).clone()
    prob.set_balance(True)
    phi1 = prob.sweep(torch.tensor(S, dtype=dt, device="cuda"))
    assert torch.equal(phi0, phi1)
    prob.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_balance_tally_of_source_iteration(api, ctx, precision, tol):
    # the tally of the returned iterate's sweep: its absorption is sigma_t
    # times the volume integral of the returned flux, and it closes
    p = inputs.random_problem((6, 5, 4), 6, 2, seed=811, c_max=0.7)
    print_case("balance_si", name=p["name"], precision=precision)
    prob = gpu_problem(api, ctx, p, precision)
    with pytest.raises(api.DgsnError, match="EINVAL"):
        prob.balance()   # nothing tallied yet
    prob.set_balance(True)
    phi, info = prob.source_iterate(tol=1e-10 if precision == "fp64" else 1e-6, max_iter=300,
                                    allow_notconv=True)
    got = prob.balance()
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    absn = (p["sigma_t"] * V * phi.double().cpu().numpy().mean(axis=2)).sum()
    scale = got["inflow"] + got["source"] + got["absorption"]
    assert abs(got["absorption"] - absn) <= tol * scale
    assert abs(got["balance"]) <= tol * scale
    prob.close()


def test_balance_tally_of_a_network_is_its_conservation_error(api, ctx, tmp_path):
    # the paper-form network does not conserve particles cell by cell; the
    # tally of its sweep is the oracle's balance of the same network sweep
    path = ARTIFACTS["paper"]
    p = inputs.random_problem((6, 5, 4), 8, 2, seed=821, length=(3.0, 2.5, 2.0))
    print_case("balance_pann", name=p["name"])
    om, w = api.quadrature_ls(8)
    prob = api.Problem(ctx, p["n"], p["length"], 2, om, w, precision="fp32", solver="ann")
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    ann = api.Ann(ctx, path)
    prob.set_ann(ann)
    prob.set_balance(True)
    S = np.repeat(p["q"][..., None], 8, axis=-1)
    prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda"))
    got = prob.balance()
    from oracle import ann_paper_train
    net = ann_paper_train.read_artifact(path)
    om_o, w_o = oracle.lq_n(8)
    mesh = (*p["n"], *p["length"])
    _, psi = oracle.pann_sweep(net, mesh, om_o, w_o, p["sigma_t"], S, p["psi_inc"],
                               store_psi=True)
    ref = oracle.sweep_balance(mesh, om_o, w_o, p["sigma_t"], S, p["psi_inc"], psi)
    scale = ref["inflow"] + ref["source"] + ref["absorption"]
    refbal = ref["outflow"] - ref["inflow"] + ref["absorption"] - ref["source"]
    assert abs(got["balance"] - refbal) <= 2e-5 * scale
    prob.close()


# ---------------------------------------------------------------------------
# non-finite iterates, expired waits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("where", ["one_cell", "everywhere"])
def test_nan_flux_is_not_reported_as_converged(api, ctx, precision, where):
    # a NaN initial guess enters the first source (sigma_s > 0) and the
    # residual: source iteration must fail with DGSN_EINVAL, never return OK
    p = inputs.random_problem((4, 4, 3), 4, 2, seed=831, c_max=0.5)
    print_case("nan_si", name=p["name"], precision=precision, where=where)
    prob = gpu_problem(api, ctx, p, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi0 = torch.zeros((2, 48, 8), dtype=dt, device="cuda")
    if where == "one_cell":
        phi0[1, 17, 3] = float("nan")
    else:
        phi0.fill_(float("nan"))
    with pytest.raises(api.DgsnError, match="DGSN_EINVAL.*non-finite"):
        prob.source_iterate(phi0=phi0, tol=1e-6, max_iter=50)
    # the problem is usable afterwards
    phi, info = prob.source_iterate(tol=1e-6, max_iter=200, allow_notconv=True)
    assert torch.isfinite(phi).all()
    prob.close()


def test_expired_wait_in_source_iteration_is_a_timeout(api, ctx):
    p = inputs.random_problem((1, 1, 64), 2, 1, seed=841, length=(0.1, 0.1, 6.4), c_max=0.5)
    print_case("si_timeout", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp32")
    prob.set_tile(1)
    prob.set_schedule("dataflow", poll_limit=1)
    with pytest.raises(api.DgsnError, match="DGSN_ETIMEOUT"):
        prob.source_iterate(tol=1e-6, max_iter=5)
    prob.set_schedule("dataflow")
    phi, info = prob.source_iterate(tol=1e-6, max_iter=200, allow_notconv=True)
    assert torch.isfinite(phi).all()
    prob.close()


# ---------------------------------------------------------------------------
# batch graphs follow their problems
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("schedule", ["planes", "dataflow"])
def test_batch_recaptures_after_problem_changes(api, ctx, schedule):
    paths = ARTIFACTS
    cases = [((6, 5, 4), 4, 2), ((5, 7, 3), 6, 1), ((4, 4, 4), 8, 2)]
    probs, srcs, phis = [], [], []
    for k, (n, order, G) in enumerate(cases):
        p = inputs.random_problem(n, order, G, seed=851 + k, length=tuple(0.2 * v for v in n))
        prob = gpu_problem(api, ctx, p, "fp32")
        probs.append(prob)
        srcs.append(torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float32,
                                 device="cuda"))
        phis.append(torch.empty_like(srcs[-1]))
    print_case("batch_recapture", schedule=schedule)
    batch = api.Batch(ctx, probs)
    for k in range(len(probs)):
        batch.set_io(k, srcs[k], phis[k])
    batch.set_schedule(schedule)
    batch.run()
    torch.cuda.synchronize()

    def check():
        for k in range(len(probs)):
            phis[k].fill_(float("nan"))
        batch.run()
        torch.cuda.synchronize()
        for k in range(len(probs)):
            ref = probs[k].sweep(srcs[k]).cpu().numpy()
            got = phis[k].cpu().numpy()
            assert rel(got, ref) <= 1e-6, k

    # a new inflow of problem 0
    probs[0].set_inflow([0.7, 0.1, 0.2, 0.9, 0.4, 0.3])
    check()
    # problem 1 switches to the paper-form network, then to another network
    pann = api.Ann(ctx, paths["paper"])
    probs[1].set_ann(pann)
    probs[1].set_solver("ann")
    check()
    mfma = api.Ann(ctx, paths["mfma"])
    probs[1].set_ann(mfma)
    check()
    # back to GE
    probs[1].set_solver("ge")
    check()
    # a member set to the dense solver is refused
    probs[2].set_solver("ge_dense")
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        batch.run()
    probs[2].set_solver("ge")
    check()
    batch.close()


# ---------------------------------------------------------------------------
# adjoint and autograd against stale state
# ---------------------------------------------------------------------------

def test_adjoint_needs_a_source_iteration_on_the_current_inputs(api, ctx):
    p = inputs.random_problem((4, 3, 3), 4, 2, seed=861, c_max=0.5)
    print_case("adjoint_state", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp64", store_psi=True)
    g = np.ones((2, 36, 8))
    with pytest.raises(api.DgsnError, match="EINVAL.*angular flux"):
        prob.adjoint(g)   # never iterated
    prob.source_iterate(tol=1e-12, max_iter=500)
    prob.adjoint(g, tol=1e-12)
    prob.adjoint(g, tol=1e-12)   # the adjoint leaves the forward state alone
    prob.set_materials(p["sigma_t"] * 1.1, p["sigma_s"], p["q"])
    with pytest.raises(api.DgsnError, match="EINVAL.*angular flux"):
        prob.adjoint(g)
    prob.source_iterate(tol=1e-12, max_iter=500)
    S = torch.ones((2, 36, 8), dtype=torch.float64, device="cuda")
    prob.sweep(S)
    with pytest.raises(api.DgsnError, match="EINVAL.*angular flux"):
        prob.adjoint(g)
    prob.close()


def test_transport_solve_backward_after_a_second_forward_raises(api, ctx):
    p = inputs.adjoint_box(n=5, groups=1, seed=871, box=(1, 3))
    print_case("autograd_state", name=p["name"])
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp64",
                       store_psi=True)
    st = torch.tensor(p["sigma_t"], device="cuda", requires_grad=True)
    q = torch.tensor(p["q"], device="cuda", requires_grad=True)
    ss = torch.tensor(p["sigma_s"], device="cuda")
    phi1 = api.TransportSolve.apply(prob, st, q, ss, 1e-12, 2000)
    phi2 = api.TransportSolve.apply(prob, st * 1.01, q, ss, 1e-12, 2000)
    with pytest.raises(RuntimeError, match="changed after this forward"):
        phi1.sum().backward()
    phi2.sum().backward()   # the latest forward is still consistent
    assert torch.isfinite(st.grad).all()
    # a forward that stops before tol warns
    with pytest.warns(RuntimeWarning, match="stopped after"):
        api.TransportSolve.apply(prob, st, q, ss, 1e-30, 3)
    prob.close()


def test_set_scattering_null_keeps_group_to_group_orders_whole(api, ctx):
    p = inputs.random_problem((3, 3, 2), 4, 2, seed=881, c_max=0.5)
    print_case("gg_null", name=p["name"])
    prob = gpu_problem(api, ctx, p, "fp64")
    mats = np.zeros((2, 2, 2, 18))
    mats[0, 0, 0] = mats[0, 1, 1] = p["sigma_s"][0].mean()
    mats[1, 0, 0] = 0.1
    prob.set_anisotropy_gg(mats)
    ref, _ = prob.source_iterate(tol=1e-12, max_iter=500)
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        prob.set_scattering(None)
    got, _ = prob.source_iterate(tol=1e-12, max_iter=500)
    assert torch.equal(got, ref)
    prob.set_anisotropy(None)   # drops orders 1..L, keeps the order-0 matrix
    prob.set_scattering(None)   # now allowed
    prob.close()

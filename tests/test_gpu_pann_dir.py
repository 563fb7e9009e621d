"""GPU parity of the paper-form networks held per quadrature direction
(version-3 artifacts) against the oracle's FP64 forward of the same stored
networks.

The per-direction kernels are the per-octant ones with each lane reading the
image of its own direction, so the tolerances are those of the per-octant
networks: FP32 forward within twice the rounding bound of one evaluation
(scaling folded into the first layer, FP32 sums, hardware exp2 and
reciprocal), and 2e-5 norm-wise for a sweep, 5e-5 for a source iteration.
Every device call goes through the C ABI.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1906_04017_amd import inputs

pytestmark = pytest.mark.gpu


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


def print_case(case, **kw):
    print(f"[case] {case} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def gpu_problem(api, ctx, p, solver="ann"):
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp32",
                       solver=solver)
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    return prob


def random_nets(seed, k, nh=8):
    """k random 26-nh-8 paper-form networks (weights of the trained nets' size)."""
    rng = np.random.default_rng(seed)
    imin, imax = np.zeros(26), np.ones(26)
    imin[12:14] = -1.0
    imax[22] = 10.0
    imin[23:26] = 0.1
    return dict(W1=rng.normal(size=(k, nh, 26)) / 5, b1=rng.normal(size=(k, nh)) / 5,
                W2=rng.normal(size=(k, 8, nh)) / 8, b2=np.abs(rng.normal(size=(k, 8))) / 5,
                imin=imin, imax=imax)


def write_dir(tmp_path, net, omega, name, perm=None):
    """Writes the version-3 artifact (nets stored in the order perm of the
    directions, if given) and returns (path, the stored networks as the
    oracle's reader sees them)."""
    from oracle import ann_paper_train
    from paper_1906_04017_amd import ann_format
    k = len(omega)
    perm = np.arange(k) if perm is None else np.asarray(perm)
    path = tmp_path / name
    ann_format.write_paper_dir(path, net["W1"][perm], net["b1"][perm], net["W2"][perm],
                               net["b2"][perm], net["imin"], net["imax"], np.asarray(omega)[perm])
    return path, ann_paper_train.read_artifact(path)


def forward_bound(net, k, I):
    """Bound on |FP32 device - FP64| for one sample of net k (see the module
    docstring)."""
    u = 2.0 ** -24
    W1, b1 = net["W1"][k].astype(np.float64), net["b1"][k].astype(np.float64)
    W2, b2 = net["W2"][k].astype(np.float64), net["b2"][k].astype(np.float64)
    c = net["alpha"] * 0.5 * (net["imin"] + net["imax"])
    r = np.abs(net["imax"] - net["imin"])
    Wf = W1 / r[None, :]
    bf = b1 - Wf @ c
    dz = 30 * u * (np.abs(Wf) @ np.abs(I) + np.abs(bf) + np.abs(Wf) @ np.abs(c))
    h = np.tanh(Wf @ I + bf)
    do = np.abs(W2) @ (dz + 2e-7) + 12 * u * (np.abs(W2) @ np.abs(h) + np.abs(b2))
    beta = net["beta_scale"] * I[:12].max()
    return max(1.0, beta) * do + 4e-7 * beta


def test_per_direction_infer_within_fp32_bound(api, ctx, tmp_path):
    om, _ = oracle.lq_n(4)
    print_case("pann_dir_infer", directions=len(om))
    path, net = write_dir(tmp_path, random_nets(600, len(om)), om, "d.dgsnann")
    ann = api.Ann(ctx, path)
    assert ann.info() == (3, 26, 8, 24)
    rng = np.random.default_rng(10)
    n = 300 + 7
    x = rng.uniform(-0.2, 1.2, size=(n, 26))
    x[:, 22] *= 10.0
    x = x.astype(np.float32)
    xd = x.astype(np.float64)
    for k in (0, 5, 11, 23):
        y = ann.infer_octant(k, torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
        for i in range(0, n, 5):
            ref = oracle.pann_forward(net, k, xd[i])
            assert np.all(np.abs(y[i] - ref) <= 2 * forward_bound(net, k, xd[i]) + 1e-7), (k, i)
    with pytest.raises(api.DgsnError, match="EINVAL"):
        ann.infer_octant(24, torch.tensor(x, device="cuda"))
    with pytest.raises(api.DgsnError, match="EINVAL"):
        ann.set_mode("bf16x2")


CASES = [((5, 4, 6), (0.5, 0.4, 0.6), 4, 2), ((7, 5, 6), (0.7, 0.5, 0.6), 6, 1),
         ((3, 8, 2), (0.3, 0.8, 0.2), 8, 3)]


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_S{c[2]}_G{c[3]}" for c in CASES])
def test_per_direction_sweep_matches_oracle(api, ctx, tmp_path, case, tile):
    n, L, order, G = case
    print_case("pann_dir_sweep", n=n, order=order, G=G, tile=tile)
    om, w = oracle.lq_n(order)
    nets = random_nets(610 + order, len(om))
    # the nets stored in a shuffled order: each direction must find its own
    perm = np.random.default_rng(order).permutation(len(om))
    path, net = write_dir(tmp_path, nets, om, "ds.dgsnann", perm=perm)
    ann = api.Ann(ctx, path)
    p = inputs.random_problem(n, order, G, seed=81 + tile, length=L)
    prob = gpu_problem(api, ctx, p)
    prob.set_ann(ann)
    prob.set_tile(tile)
    rng = np.random.default_rng(17)
    S = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1) +
                     rng.uniform(-0.2, 0.5, size=(G, p["sigma_t"].shape[1], 8)),
                     dtype=torch.float32, device="cuda")
    phi = prob.sweep(S).clone()
    ref = oracle.pann_sweep(net, mesh_of(p), om, w, p["sigma_t"], S.cpu().numpy(), p["psi_inc"])
    assert rel(phi.cpu().numpy(), ref) <= 2e-5
    # the same networks as a per-octant sweep would give something else: the
    # per-direction images are in use
    from paper_1906_04017_amd import ann_format
    po = tmp_path / "po.dgsnann"
    ann_format.write_paper(po, nets["W1"][:8], nets["b1"][:8], nets["W2"][:8], nets["b2"][:8],
                           nets["imin"], nets["imax"])
    ann_o = api.Ann(ctx, po)
    prob.set_ann(ann_o)
    other = prob.sweep(S).cpu().numpy()
    assert rel(other, ref) > 1e-3
    prob.set_ann(ann)
    # the dataflow schedule runs the same arithmetic
    prob.set_schedule("dataflow")
    for _ in range(2):
        got = prob.sweep(S)
        prob.check()
        assert torch.equal(got, phi)


def test_per_direction_source_iteration_matches_oracle(api, ctx, tmp_path):
    om, w = oracle.lq_n(4)
    path, net = write_dir(tmp_path, random_nets(620, len(om)), om, "dsi.dgsnann")
    ann = api.Ann(ctx, path)
    p = inputs.random_problem((6, 5, 4), 4, 2, seed=91, c_max=0.5, length=(0.6, 0.5, 0.4))
    print_case("pann_dir_si", name=p["name"])
    prob = gpu_problem(api, ctx, p)
    prob.set_ann(ann)
    phi, info = prob.source_iterate(tol=1e-6, max_iter=200)
    ref = oracle.pann_source_iterate(net, mesh_of(p), om, w, p["sigma_t"], p["sigma_s"], p["q"],
                                     p["psi_inc"], tol=1e-10, max_iter=500)
    assert rel(phi.cpu().numpy(), ref["phi"]) <= 5e-5


def test_per_direction_attach_and_batch_rules(api, ctx, tmp_path):
    om4, _ = oracle.lq_n(4)
    path, _ = write_dir(tmp_path, random_nets(630, len(om4)), om4, "dr.dgsnann")
    ann = api.Ann(ctx, path)
    # an S6 problem has directions the S4 artifact does not hold: refused,
    # and the network attached before stays in use
    p6 = inputs.random_problem((4, 4, 3), 6, 1, seed=92)
    print_case("pann_dir_rules", name=p6["name"])
    om6, _ = oracle.lq_n(6)
    path6, _ = write_dir(tmp_path, random_nets(631, len(om6)), om6, "d6.dgsnann")
    ann6 = api.Ann(ctx, path6)
    prob = gpu_problem(api, ctx, p6)
    prob.set_ann(ann6)
    S = torch.ones((1, p6["sigma_t"].shape[1], 8), dtype=torch.float32, device="cuda")
    good = prob.sweep(S).cpu().numpy()
    with pytest.raises(api.DgsnError, match="EINVAL.*no network"):
        prob.set_ann(ann)
    assert np.array_equal(prob.sweep(S).cpu().numpy(), good)
    # batches take per-octant networks only
    batch = api.Batch(ctx, [prob])
    phi = torch.zeros_like(S)
    batch.set_io(0, S, phi)
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED"):
        batch.run()
    batch.close()
    # FP32 forward sweeps only
    p4 = inputs.random_problem((3, 3, 3), 4, 1, seed=93)
    om, w = api.quadrature_ls(4)
    prob64 = api.Problem(ctx, p4["n"], p4["length"], 1, om, w, precision="fp64")
    with pytest.raises(api.DgsnError):
        prob64.set_ann(ann)


def test_per_direction_refuses_more_directions_than_lds_holds(api, ctx, tmp_path):
    # a sweep block holds its octant's per-direction images in 64 KB of LDS
    # (59 directions per octant): a 60-direction-per-octant set is refused
    rng = np.random.default_rng(640)
    base = np.abs(rng.normal(size=(60, 3)))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    signs = [np.array([-1.0 if (o >> a) & 1 else 1.0 for a in range(3)]) for o in range(8)]
    om = np.concatenate([base * s for s in signs])
    w = np.full(len(om), 4.0 * np.pi / len(om))
    print_case("pann_dir_lds_limit", directions=len(om))
    path, _ = write_dir(tmp_path, random_nets(641, len(om)), om, "dl.dgsnann")
    ann = api.Ann(ctx, path)
    prob = api.Problem(ctx, (2, 2, 2), (1.0, 1.0, 1.0), 1, om, w, precision="fp32",
                       solver="ann")
    with pytest.raises(api.DgsnError, match="EUNSUPPORTED.*59"):
        prob.set_ann(ann)

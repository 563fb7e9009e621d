"""Offline training of the paper-form shallow ANN (Sec. 3 and the training
paragraphs of Sec. 4) -- TEST INFRASTRUCTURE / artifact generator.

Writes the per-octant network artifact consumed by the library
(dgsn_ann_load, version 2).  It calls only the oracle: the training targets
are FP64 one-cell solutions obtained by assembly + Gaussian elimination in the
physical orientation (oracle.cell_solve_batch).

Network (Sec. 3): 26 inputs in the physical frame of the cell, in the order
the paper lists them (12 inflow face values, the two direction cosines
omega_x, omega_y, 8 nodal source values, sigma_t, dx, dy, dz; the layout is
oracle.pann_inputs), each scaled by Eq. (ANN:Eq2) with alpha = 0.27 and the
sampling bounds as I_min / I_max; one hidden layer of 8 tanh units
(Eq. (ANN:Eq3)); 8 outputs through the ELU of Eq. (ANN:Eq4) with
beta = 0.1 max(psi_inc) per sample.  One network per octant (first
paragraphs of Sec. 4), each trained on 9e4 problems of its octant and tested
on 1e4 more.

Loss: Eq. (Test:Eq1), the mean absolute error plus the regulariser on the
error of the node sum relative to the solution size, lambda = 0.2,
gamma_1 = 10, gamma_2 = 0.01.  Optimiser: Adam (the paper uses learning rates
in [5e-5, 2e-4] for 5e4 epochs; here a cosine schedule from 2e-3 down to 5e-5
over far fewer mini-batch epochs reaches its plateau on a CPU).

Connection pruning (the paper's "dropout" paragraph of Sec. 3): repeatedly
drop the connection (a W1 or W2 entry) of smallest magnitude, retrain the
remaining ones briefly, and stop when the training mean squared error has
grown by more than 0.1 % over that of the unpruned network (the last drop is
then undone).  Dropped connections are stored as exact zeros.

Sampling (the paper samples uniformly and does not state the ranges; these
are the reading used here, see the design notes): direction uniform on the
octant's part of the unit sphere; inflow values U[0, 1] per face node;
nodal sources U[0, 1]; sigma_t U[0, 10]; dx, dy, dz U[0.1, 1] independently
(a 10 cm cube cut into 10 to 100 cells per axis).  These bounds are the
I_min / I_max of the scaling (omega_x and omega_y use [-1, 1], as the paper gives).

Per-direction networks (--per-direction; the reading of the training
paragraph of Sec. 4 that trains an ANN for each direction): one network per
direction of the LQ_N quadrature, each trained at one problem's sigma_t and
cell size (the problem's conditions held fixed, the inflow and the sources
sampled by sample_direction), written as the version-3 artifact.

Usage: python -m oracle.ann_paper_train --out paper_1906_04017_amd/data/ann_paper_tanh8.dgsnann
       python -m oracle.ann_paper_train --per-direction --order 8 --sigma-t 10 --h 0.1 \
           --out paper_1906_04017_amd/data/ann_paper_dir_s8_sig10_h0.1.dgsnann
"""
import argparse
import struct
import time
import zlib

import numpy as np
import torch

import oracle

LAMBDA, GAMMA1, GAMMA2 = 0.2, 10.0, 0.01
ALPHA, BETA_SCALE = 0.27, 0.1
PSI_MAX, S_MAX, SIG_MAX, H_MIN, H_MAX = 1.0, 1.0, 10.0, 0.1, 1.0


def octant_signs(o):
    return np.array([-1.0 if (o >> a) & 1 else 1.0 for a in range(3)])


def bounds(psi_max=PSI_MAX, s_max=S_MAX):
    """I_min, I_max of the 26 inputs (the same for every octant; the paper
    gives (mu, eta) in [-1, 1])."""
    imin = np.zeros(26)
    imax = np.zeros(26)
    imax[0:12] = psi_max
    imin[12:14], imax[12:14] = -1.0, 1.0
    imax[14:22] = s_max
    imax[22] = SIG_MAX
    imin[23:26], imax[23:26] = H_MIN, H_MAX
    return imin, imax


def sample(n, o, rng):
    """n random one-cell problems of octant o: raw inputs I [n, 26] and the
    FP64 assembly + GE solutions psi [n, 8] (physical node order)."""
    sg = octant_signs(o)
    om = np.abs(rng.normal(size=(n, 3)))
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    om *= sg[None, :]
    h = rng.uniform(H_MIN, H_MAX, size=(n, 3))
    sig = rng.uniform(0.0, SIG_MAX, size=n)
    S = rng.uniform(0.0, S_MAX, size=(n, 8))
    face = rng.uniform(0.0, PSI_MAX, size=(n, 3, 4))
    up = np.zeros((n, 6, 8))
    for a in range(3):
        side = 1 if sg[a] < 0 else 0
        t1, t2 = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
        for fn in range(4):
            node = (side << a) | ((fn & 1) << t1) | (((fn >> 1) & 1) << t2)
            up[:, 2 * a + side, node] = face[:, a, fn]
    psi = oracle.cell_solve_batch(h, om, sig, S, up)
    I = np.concatenate([face.reshape(n, 12), om[:, :2], S, sig[:, None], h], axis=1)
    return I, psi


def sample_direction(n, omega, sigma_t, h, rng, recipe="uniform", psi_max=PSI_MAX,
                     s_max=S_MAX):
    """n random one-cell problems of one direction at a fixed sigma_t and
    cell size h [3]: raw inputs I [n, 26] and the FP64 assembly + GE
    solutions psi [n, 8].  recipe "uniform": inflow U[0, 1] per face node,
    sources U[0, 1] per node (the per-octant recipe with the direction,
    sigma_t and cell fixed); "smooth": 90 % of the inflow faces a level
    U[0, 1] with a bilinear tilt of +-0.15 per tangential axis (clipped at 0),
    10 % U[0, 1] per node; sources zero, a constant U[0, 1] or U[0, 1] per node
    (a third each).  The inflow values are then scaled by psi_max and the
    sources by s_max (the ranges of the problem's fluxes and sources)."""
    om = np.asarray(omega, np.float64)
    sg = np.where(om < 0, -1.0, 1.0)
    hh = np.tile(np.asarray(h, np.float64), (n, 1))
    sig = np.full(n, float(sigma_t))
    if recipe == "uniform":
        S = rng.uniform(0.0, S_MAX, size=(n, 8))
        face = rng.uniform(0.0, PSI_MAX, size=(n, 3, 4))
    elif recipe == "smooth":
        kind = rng.integers(0, 3, size=(n, 1))
        level = rng.uniform(0.0, S_MAX, size=(n, 1))
        S = np.where(kind == 0, 0.0, np.where(kind == 1, level, rng.uniform(0.0, S_MAX, (n, 8))))
        lvl = rng.uniform(0.0, PSI_MAX, size=(n, 3, 1))
        tilt = rng.uniform(-0.15, 0.15, size=(n, 3, 2))
        fn = np.arange(4)
        smooth = lvl + tilt[:, :, :1] * (2.0 * (fn & 1) - 1.0) + \
            tilt[:, :, 1:] * (2.0 * ((fn >> 1) & 1) - 1.0)
        rough = rng.uniform(size=(n, 1, 1)) < 0.1
        face = np.where(rough, rng.uniform(0.0, PSI_MAX, size=(n, 3, 4)),
                        np.clip(smooth, 0.0, PSI_MAX))
    else:
        raise ValueError(f"unknown recipe {recipe}")
    face = face * (psi_max / PSI_MAX)
    S = S * (s_max / S_MAX)
    up = np.zeros((n, 6, 8))
    for a in range(3):
        side = 1 if sg[a] < 0 else 0
        t1, t2 = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
        for f in range(4):
            node = (side << a) | ((f & 1) << t1) | (((f >> 1) & 1) << t2)
            up[:, 2 * a + side, node] = face[:, a, f]
    oms = np.tile(om, (n, 1))
    psi = oracle.cell_solve_batch(hh, oms, sig, S, up)
    I = np.concatenate([face.reshape(n, 12), oms[:, :2], S, sig[:, None], hh], axis=1)
    return I, psi


class PaperNet(torch.nn.Module):
    """Eq. (ANN:Eq1)-(ANN:Eq4) on scaled inputs, with connection masks."""

    def __init__(self, nh, imin, imax):
        super().__init__()
        self.l1 = torch.nn.Linear(26, nh)
        self.l2 = torch.nn.Linear(nh, 8)
        self.register_buffer("c", torch.tensor(ALPHA * 0.5 * (imin + imax)))
        self.register_buffer("r", torch.tensor(np.abs(imax - imin)))
        self.register_buffer("m1", torch.ones(nh, 26, dtype=torch.float64))
        self.register_buffer("m2", torch.ones(8, nh, dtype=torch.float64))

    def forward(self, I):
        x = (I - self.c) / self.r
        h = torch.tanh(torch.nn.functional.linear(x, self.l1.weight * self.m1, self.l1.bias))
        z = torch.nn.functional.linear(h, self.l2.weight * self.m2, self.l2.bias)
        beta = BETA_SCALE * I[:, :12].max(dim=1, keepdim=True).values
        return torch.where(z >= 0, z, beta * (torch.exp(torch.clamp(z, max=0.0)) - 1.0))


def loss_fn(pred, y):
    mae = (pred - y).abs().mean()
    reg = ((y - pred).sum(1).abs() / (GAMMA1 * y.sum(1).abs() + GAMMA2)).mean()
    return mae + LAMBDA * reg


def fit(net, X, Y, epochs, lr0, lr1, batch=256, gen=None):
    opt = torch.optim.Adam(net.parameters(), lr=lr0)
    steps = epochs * ((len(X) + batch - 1) // batch)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=max(steps, 1), eta_min=lr1)
    for _ in range(epochs):
        perm = torch.randperm(len(X), generator=gen)
        for i in range(0, len(X), batch):
            idx = perm[i:i + batch]
            opt.zero_grad()
            loss_fn(net(X[idx]), Y[idx]).backward()
            opt.step()
            sched.step()


def mse(net, X, Y):
    with torch.no_grad():
        return float(((net(X) - Y) ** 2).mean())


def train_octant(o, nh=8, n_train=90_000, n_test=10_000, epochs=60, prune_epochs=1,
                 max_drops=80, seed=3, log=print):
    rng = np.random.default_rng([seed, o])
    gen = torch.Generator().manual_seed(seed * 8 + o)
    torch.manual_seed(seed * 8 + o)
    imin, imax = bounds()
    I, psi = sample(n_train + n_test, o, rng)
    X = torch.tensor(I[:n_train])
    Y = torch.tensor(psi[:n_train])
    Xt = torch.tensor(I[n_train:])
    Yt = torch.tensor(psi[n_train:])
    net = PaperNet(nh, imin, imax).double()
    t0 = time.time()
    fit(net, X, Y, epochs, 2e-3, 5e-5, gen=gen)
    base = mse(net, X, Y)
    log(f"octant {o}: trained in {time.time() - t0:.0f} s, train MSE {base:.3e}, "
        f"test MSE {mse(net, Xt, Yt):.3e}")
    # magnitude pruning with retraining, stopped at a 0.1 % rise of the training MSE
    drops = 0
    while drops < max_drops:
        saved = {k: v.clone() for k, v in net.state_dict().items()}
        w1 = (net.l1.weight.detach().abs() + (1 - net.m1) * 1e30).flatten()
        w2 = (net.l2.weight.detach().abs() + (1 - net.m2) * 1e30).flatten()
        if float(torch.min(w1)) <= float(torch.min(w2)):
            net.m1.view(-1)[int(torch.argmin(w1))] = 0.0
        else:
            net.m2.view(-1)[int(torch.argmin(w2))] = 0.0
        fit(net, X, Y, prune_epochs, 2e-4, 5e-5, gen=gen)
        if mse(net, X, Y) > base * 1.001:
            net.load_state_dict(saved)
            break
        drops += 1
    W1 = (net.l1.weight * net.m1).detach().numpy()
    W2 = (net.l2.weight * net.m2).detach().numpy()
    with torch.no_grad():
        e = (net(Xt) - Yt).abs()
        etr = (net(X) - Y).abs()
    st = dict(octant=o, connections=int(net.m1.sum() + net.m2.sum()), dropped=drops,
              train_mae=float(etr.mean()), train_max=float(etr.max()),
              test_mse=float((e ** 2).mean()), test_max=float(e.max()))
    log(f"octant {o}: {drops} connections dropped ({st['connections']} left); train MAE "
        f"{st['train_mae']:.3e} max {st['train_max']:.3e}; test MSE {st['test_mse']:.3e} "
        f"max {st['test_max']:.3e}")
    return W1, net.l1.bias.detach().numpy(), W2, net.l2.bias.detach().numpy(), imin, imax, st


def _train_one(o, **kw):
    torch.set_num_threads(1)
    return train_octant(o, log=lambda m: print(m, flush=True), **kw)


def train_direction(k, omega, sigma_t, h, nh=8, n_train=90_000, n_test=10_000, epochs=60,
                    seed=3, recipe="uniform", psi_max=PSI_MAX, s_max=S_MAX):
    """Network of quadrature direction k (cosines omega) at a fixed sigma_t
    and cell size h, on 9e4 + 1e4 problems of sample_direction (inflow and
    source ranges psi_max, s_max, which are also the scaling bounds); not
    pruned."""
    torch.set_num_threads(1)
    rng = np.random.default_rng([seed, 1000 + k])
    gen = torch.Generator().manual_seed(seed * 4096 + k)
    torch.manual_seed(seed * 4096 + k)
    imin, imax = bounds(psi_max, s_max)
    I, psi = sample_direction(n_train + n_test, omega, sigma_t, h, rng, recipe, psi_max, s_max)
    X, Y = torch.tensor(I[:n_train]), torch.tensor(psi[:n_train])
    Xt, Yt = torch.tensor(I[n_train:]), torch.tensor(psi[n_train:])
    net = PaperNet(nh, imin, imax).double()
    fit(net, X, Y, epochs, 2e-3, 5e-5, gen=gen)
    with torch.no_grad():
        e = (net(Xt) - Yt).abs()
        etr = (net(X) - Y).abs()
        bias = float((net(Xt) - Yt).mean())
    st = dict(direction=k, omega=[round(float(v), 6) for v in omega],
              train_mae=float(etr.mean()), train_max=float(etr.max()),
              test_mse=float((e ** 2).mean()), test_max=float(e.max()), test_bias=bias)
    print(f"direction {k}: train MAE {st['train_mae']:.3e} max {st['train_max']:.3e}; test MSE "
          f"{st['test_mse']:.3e} max {st['test_max']:.3e}", flush=True)
    return (net.l1.weight.detach().numpy(), net.l1.bias.detach().numpy(),
            net.l2.weight.detach().numpy(), net.l2.bias.detach().numpy(), imin, imax, st)


def _train_dir(args, **kw):
    k, omega = args
    return train_direction(k, omega, **kw)


def write_artifact(path, nets, alpha=ALPHA, beta_scale=BETA_SCALE):
    """Version-2 artifact: per-octant paper-form networks (same container as
    the version-1 file: magic, header words, float32 payload, CRC-32)."""
    nh = nets[0][0].shape[0]
    imin, imax = nets[0][4], nets[0][5]
    body = b"DGSNANN1" + struct.pack("<7I", 2, 26, nh, 8, 1, 1, 8)
    body += struct.pack("<2f", alpha, beta_scale)
    body += np.asarray(imin, "<f4").tobytes() + np.asarray(imax, "<f4").tobytes()
    for W1, b1, W2, b2, *_ in nets:
        for a in (W1, b1, W2, b2):
            body += np.ascontiguousarray(a, "<f4").tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def write_artifact_dir(path, nets, omega, alpha=ALPHA, beta_scale=BETA_SCALE):
    """Version-3 artifact: one paper-form network per quadrature direction,
    net k serving direction omega[k] (the version-2 header, then the
    directions as float32 [K][3], then the K networks)."""
    nh = nets[0][0].shape[0]
    imin, imax = nets[0][4], nets[0][5]
    omega = np.asarray(omega, np.float64).reshape(len(nets), 3)
    body = b"DGSNANN1" + struct.pack("<7I", 3, 26, nh, 8, 1, 1, len(nets))
    body += struct.pack("<2f", alpha, beta_scale)
    body += np.asarray(imin, "<f4").tobytes() + np.asarray(imax, "<f4").tobytes()
    body += np.ascontiguousarray(omega, "<f4").tobytes()
    for W1, b1, W2, b2, *_ in nets:
        for a in (W1, b1, W2, b2):
            body += np.ascontiguousarray(a, "<f4").tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def read_artifact(path):
    """Oracle-side reader of the version-2 (per octant) and version-3 (per
    direction, with the directions under "omega") artifacts -> oracle.pann_*
    net dict."""
    data = open(path, "rb").read()
    if data[:8] != b"DGSNANN1":
        raise ValueError("bad magic")
    ver, nin, nh, nout, act, flags, nnet = struct.unpack("<7I", data[8:36])
    if ver not in (2, 3) or nin != 26 or nout != 8 or (ver == 2 and nnet != 8):
        raise ValueError("not a paper-form (version 2 or 3) artifact")
    if struct.unpack("<I", data[-4:])[0] != zlib.crc32(data[:-4]) & 0xFFFFFFFF:
        raise ValueError("checksum mismatch")
    alpha, beta_scale = struct.unpack("<2f", data[36:44])
    f = np.frombuffer(data[44:-4], dtype="<f4").astype(np.float64)
    imin, imax = f[:26], f[26:52]
    o = 52
    omega = None
    if ver == 3:
        omega = f[o:o + 3 * nnet].reshape(nnet, 3)
        o += 3 * nnet
    W1, b1, W2, b2 = [], [], [], []
    for _ in range(nnet):
        W1.append(f[o:o + nh * 26].reshape(nh, 26)); o += nh * 26
        b1.append(f[o:o + nh]); o += nh
        W2.append(f[o:o + 8 * nh].reshape(8, nh)); o += 8 * nh
        b2.append(f[o:o + 8]); o += 8
    net = dict(kind="paper", W1=np.array(W1), b1=np.array(b1), W2=np.array(W2),
               b2=np.array(b2), imin=imin, imax=imax, alpha=float(alpha),
               beta_scale=float(beta_scale))
    if omega is not None:
        net["omega"] = omega
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--hidden", type=int, default=8)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--max-drops", type=int, default=80)
    ap.add_argument("--per-direction", action="store_true",
                    help="one network per direction of the LQ_N quadrature (version 3)")
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--sigma-t", type=float, default=10.0)
    ap.add_argument("--h", type=float, default=0.1, help="cell edge (cubic cells)")
    ap.add_argument("--recipe", default="smooth", choices=("uniform", "smooth"))
    ap.add_argument("--psi-max", type=float, default=PSI_MAX,
                    help="range of the inflow values (per-direction networks)")
    ap.add_argument("--s-max", type=float, default=S_MAX,
                    help="range of the nodal sources (per-direction networks)")
    a = ap.parse_args()
    # one process per network, one thread each (the networks are tiny)
    import concurrent.futures
    import functools
    if a.per_direction:
        omega, _ = oracle.lq_n(a.order)
        job = functools.partial(_train_dir, sigma_t=a.sigma_t, h=(a.h,) * 3, nh=a.hidden,
                                epochs=a.epochs, seed=a.seed, recipe=a.recipe,
                                psi_max=a.psi_max, s_max=a.s_max)
        with concurrent.futures.ProcessPoolExecutor(max_workers=max(1, a.threads)) as ex:
            nets = list(ex.map(job, list(enumerate(omega))))
        write_artifact_dir(a.out, nets, omega)
        print(f"wrote {a.out}")
        for n in nets:
            print(n[-1])
        return
    job = functools.partial(_train_one, nh=a.hidden, epochs=a.epochs, seed=a.seed,
                            max_drops=a.max_drops)
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(8, a.threads)) as ex:
        nets = list(ex.map(job, range(8)))
    write_artifact(a.out, nets)
    print(f"wrote {a.out}")
    for n in nets:
        print(n[-1])


if __name__ == "__main__":
    main()

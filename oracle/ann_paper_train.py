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

Usage: python -m oracle.ann_paper_train --out paper_1906_04017_amd/data/ann_paper_tanh8.dgsnann
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


def bounds():
    """I_min, I_max of the 26 inputs (the same for every octant; the paper
    gives (mu, eta) in [-1, 1])."""
    imin = np.zeros(26)
    imax = np.zeros(26)
    imax[0:12] = PSI_MAX
    imin[12:14], imax[12:14] = -1.0, 1.0
    imax[14:22] = S_MAX
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


def read_artifact(path):
    """Oracle-side reader of the version-2 artifact -> oracle.pann_* net dict."""
    data = open(path, "rb").read()
    if data[:8] != b"DGSNANN1":
        raise ValueError("bad magic")
    ver, nin, nh, nout, act, flags, nnet = struct.unpack("<7I", data[8:36])
    if ver != 2 or nin != 26 or nout != 8 or nnet != 8:
        raise ValueError("not a version-2 paper-form artifact")
    if struct.unpack("<I", data[-4:])[0] != zlib.crc32(data[:-4]) & 0xFFFFFFFF:
        raise ValueError("checksum mismatch")
    alpha, beta_scale = struct.unpack("<2f", data[36:44])
    f = np.frombuffer(data[44:-4], dtype="<f4").astype(np.float64)
    imin, imax = f[:26], f[26:52]
    o = 52
    W1, b1, W2, b2 = [], [], [], []
    for _ in range(8):
        W1.append(f[o:o + nh * 26].reshape(nh, 26)); o += nh * 26
        b1.append(f[o:o + nh]); o += nh
        W2.append(f[o:o + 8 * nh].reshape(8, nh)); o += 8 * nh
        b2.append(f[o:o + 8]); o += 8
    return dict(kind="paper", W1=np.array(W1), b1=np.array(b1), W2=np.array(W2),
                b2=np.array(b2), imin=imin, imax=imax, alpha=float(alpha),
                beta_scale=float(beta_scale))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--hidden", type=int, default=8)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--max-drops", type=int, default=80)
    a = ap.parse_args()
    # one process per octant network, one thread each (the networks are tiny)
    import concurrent.futures
    import functools
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

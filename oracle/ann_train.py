"""Offline training of the shallow ANN local solver (Sec. 3 and the training
paragraphs of Sec. 4) -- TEST INFRASTRUCTURE / artifact generator.

Writes the network artifact consumed by the library (dgsn_ann_load).  It
calls only the oracle: training targets are FP64 one-cell solutions of the
canonical cell system obtained by assembly + Gaussian elimination
(oracle.cell_solve_batch), as the paper generates its training sets from
solved random one-cell problems.

Network: 24 inputs (the reduced one-cell parametrisation of Sec. 3 in the
canonical octant: streaming weights kappa_a h, optical size sigma_t h, the 12
inflow face values and 8 source nodes, the last 20 divided by the homogeneity
scale m), one hidden layer of 64 ReLU units, 8 linear outputs = psi / m.
Loss: the paper's mean absolute error plus the regulariser that penalises the
error of the node sum relative to the solution size (Eq. (Test:Eq1),
lambda = 0.2, gamma_1 = 10, gamma_2 = 0.01).  Optimiser: Adam.

Sampling (the paper samples uniformly but does not give ranges):
  directions: the canonical-octant directions of the LQ_N set the artifact
  serves (--order; the paper trains one net per octant, here every octant is
  reflected onto the canonical one), or uniform on the octant sphere
  (--order 0); cubic cells;
  tau = sigma_t h log-uniform on [1e-5, 4];
  inflow faces: 90 % smooth (per-face level U[0, 1] plus a small bilinear
  variation), 10 % independent U[-0.1, 1] node values;
  sources h S = tau U[0, 2] (1 + U[-0.3, 0.3] per node); 10 % pure-inflow and
  10 % pure-source problems.

Usage: python -m oracle.ann_train --out paper_1906_04017_amd/data/ann_relu64.dgsnann
"""
import argparse
import struct
import time
import zlib

import numpy as np
import torch

import oracle

LAMBDA, GAMMA1, GAMMA2 = 0.2, 10.0, 0.01


def sample_problems(n, seed, order=None, rough=0.1):
    rng = np.random.default_rng(seed)
    om = np.abs(rng.normal(size=(n, 3)))
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    if order:
        # directions of the canonical octant of the LQ_N set the net serves
        oq, _ = oracle.lq_n(order)
        oq = oq[:len(oq) // 8]
        om = oq[rng.integers(0, len(oq), size=n)]
    tau = 10.0 ** rng.uniform(-5.0, np.log10(4.0), size=n)
    pin = np.empty((n, 12))
    smooth = rng.uniform(size=n) >= rough
    lev = rng.uniform(0.0, 1.0, size=(n, 3, 1))
    grad = rng.uniform(-0.15, 0.15, size=(n, 3, 2))
    fn = np.arange(4)
    bil = lev + grad[:, :, :1] * (fn & 1)[None, None, :] + grad[:, :, 1:] * (fn >> 1)[None, None, :]
    pin[smooth] = bil[smooth].reshape(-1, 12)
    pin[~smooth] = rng.uniform(-0.1, 1.0, size=(int((~smooth).sum()), 12))
    hs = tau[:, None] * rng.uniform(0.0, 2.0, size=(n, 1)) * (1 + rng.uniform(-0.3, 0.3, (n, 8)))
    kind = rng.uniform(size=n)
    pin[kind < 0.1] = 0.0
    hs[(kind >= 0.1) & (kind < 0.2)] = 0.0
    return om, tau, pin, hs


def solve_targets(om, tau, pin, hs, h=1.0):
    """FP64 assembly + GE of each canonical cell (unit cube, all components >= 0)."""
    n = om.shape[0]
    up = np.zeros((n, 6, 8))
    for fn in range(4):
        up[:, 0, 2 * fn] = pin[:, fn]
        up[:, 2, (fn & 1) + 4 * (fn >> 1)] = pin[:, 4 + fn]
        up[:, 4, fn] = pin[:, 8 + fn]
    return oracle.cell_solve_batch(np.full(3, h), om, tau / h, hs / h, up)


def features(om, tau, pin, hs):
    """24 normalised inputs and the scale m (same definition as the oracle's
    ANN sweep, orc_ann_features, for cubic cells)."""
    kmax = om.max(axis=1)
    m = np.maximum(np.abs(pin).max(axis=1), np.abs(hs).max(axis=1) / (tau + kmax))
    ms = np.where(m > 0, m, 1.0)
    x = np.concatenate([om, tau[:, None], pin / ms[:, None], hs / ms[:, None]], axis=1)
    return x, m


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def write_artifact(path, W1, b1, W2, b2, act=0):
    W1, b1, W2, b2 = (np.ascontiguousarray(a, dtype="<f4") for a in (W1, b1, W2, b2))
    nh, nin = W1.shape
    body = b"DGSNANN1" + struct.pack("<6I", 1, nin, nh, W2.shape[0], act, 0)
    body += W1.tobytes() + b1.tobytes() + W2.tobytes() + b2.tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def read_artifact(path):
    data = open(path, "rb").read()
    if data[:8] != b"DGSNANN1":
        raise ValueError("bad magic")
    ver, nin, nh, nout, act, flags = struct.unpack("<6I", data[8:32])
    if struct.unpack("<I", data[-4:])[0] != zlib.crc32(data[:-4]) & 0xFFFFFFFF:
        raise ValueError("checksum mismatch")
    f = np.frombuffer(data[32:-4], dtype="<f4").astype(np.float64)
    o = 0
    W1 = f[o:o + nh * nin].reshape(nh, nin); o += nh * nin
    b1 = f[o:o + nh]; o += nh
    W2 = f[o:o + nout * nh].reshape(nout, nh); o += nout * nh
    b2 = f[o:o + nout]
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, act=act)


def loss_fn(pred, y):
    mae = (pred - y).abs().mean()
    reg = ((y - pred).sum(1).abs() / (GAMMA1 * y.sum(1).abs() + GAMMA2)).mean()
    return mae + LAMBDA * reg


def train(n_train=1_000_000, n_test=20_000, hidden=64, epochs=40, batch=2048, lr=2e-3, seed=3,
          threads=8, order=8, log=print):
    torch.manual_seed(seed)
    torch.set_num_threads(threads)
    om, tau, pin, hs = sample_problems(n_train + n_test, seed, order=order)
    t0 = time.time()
    psi = solve_targets(om, tau, pin, hs)
    x, m = features(om, tau, pin, hs)
    ms = np.where(m > 0, m, 1.0)
    y = psi / ms[:, None]
    log(f"targets: {len(x)} one-cell GE solves in {time.time() - t0:.1f} s")
    X = torch.tensor(x[:n_train], dtype=torch.float32)
    Y = torch.tensor(y[:n_train], dtype=torch.float32)
    Xt = torch.tensor(x[n_train:], dtype=torch.float32)
    Yt = torch.tensor(y[n_train:], dtype=torch.float32)
    net = torch.nn.Sequential(torch.nn.Linear(24, hidden), torch.nn.ReLU(),
                              torch.nn.Linear(hidden, 8))
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=epochs, eta_min=lr * 0.02)
    for ep in range(epochs):
        perm = torch.randperm(n_train)
        tot = 0.0
        for i in range(0, n_train, batch):
            idx = perm[i:i + batch]
            opt.zero_grad()
            loss = loss_fn(net(X[idx]), Y[idx])
            loss.backward()
            opt.step()
            tot += float(loss) * len(idx)
        sched.step()
        with torch.no_grad():
            e = (net(Xt) - Yt).abs()
        log(f"epoch {ep + 1}/{epochs} loss {tot / n_train:.3e} test MAE {float(e.mean()):.3e} "
            f"max {float(e.max()):.3e}")
    W1 = net[0].weight.detach().numpy()
    b1 = net[0].bias.detach().numpy()
    W2 = net[2].weight.detach().numpy()
    b2 = net[2].bias.detach().numpy()
    # weights stored BF16-exact (the matrix cores consume BF16); biases FP32
    W1q, W2q = bf16_round(W1), bf16_round(W2)
    with torch.no_grad():
        net[0].weight.copy_(torch.tensor(W1q))
        net[2].weight.copy_(torch.tensor(W2q))
        e = (net(Xt) - Yt).abs()
    stats = dict(test_mae=float(e.mean()), test_max=float(e.max()),
                 test_mse=float((e ** 2).mean()))
    log(f"after BF16 weight rounding: test MAE {stats['test_mae']:.3e} max {stats['test_max']:.3e}")
    return W1q, b1, W2q, b2, stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-train", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--order", type=int, default=8)
    a = ap.parse_args()
    W1, b1, W2, b2, stats = train(n_train=a.n_train, hidden=a.hidden, epochs=a.epochs,
                                  seed=a.seed, threads=a.threads, order=a.order)
    write_artifact(a.out, W1, b1, W2, b2)
    print(f"wrote {a.out}: {stats}")


if __name__ == "__main__":
    main()

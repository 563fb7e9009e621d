"""Writer/reader of the shallow-ANN artifacts consumed by dgsn_ann_load.

Version 1 (the canonical 24-input network on the matrix cores), little
endian: b"DGSNANN1", u32 version=1, u32 n_in=24, u32 n_hidden, u32 n_out=8,
u32 activation (0 = ReLU, 1 = tanh), u32 flags, float32 W1[n_hidden][n_in],
b1[n_hidden], W2[n_out][n_hidden], b2[n_out], u32 CRC-32 (IEEE) of all
preceding bytes.

Version 2 (the paper-form networks, one per octant): b"DGSNANN1", u32
version=2, u32 n_in=26, u32 n_hidden, u32 n_out=8, u32 activation=1 (tanh),
u32 flags=1 (ELU output), u32 n_nets=8, float32 alpha, float32 beta_scale,
float32 imin[26], float32 imax[26], then per octant 0..7 float32
W1[n_hidden][26], b1[n_hidden], W2[8][n_hidden], b2[8], then the CRC-32.

Version 3 (the paper-form networks, one per quadrature direction): the
version-2 layout with version=3 and n_nets = K, float32 omega[K][3] after
imax, then the K networks in the order of omega.
"""
import struct
import zlib

import numpy as np

MAGIC = b"DGSNANN1"


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    return a.reshape(shape) if shape is not None else a


def write(path, W1, b1, W2, b2, activation=0, flags=0):
    W1 = _f32(W1)
    b1 = _f32(b1).reshape(-1)
    W2 = _f32(W2)
    b2 = _f32(b2).reshape(-1)
    nh, nin = W1.shape
    nout = W2.shape[0]
    if W2.shape != (nout, nh) or b1.shape != (nh,) or b2.shape != (nout,):
        raise ValueError("inconsistent ANN parameter shapes")
    body = MAGIC + struct.pack("<6I", 1, nin, nh, nout, int(activation), int(flags))
    body += W1.tobytes() + b1.tobytes() + W2.tobytes() + b2.tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def write_paper(path, W1, b1, W2, b2, imin, imax, alpha=0.27, beta_scale=0.1, n_in=26,
                activation=1, flags=1):
    """Version-2 artifact: W1 [8][nh][26], b1 [8][nh], W2 [8][8][nh], b2 [8][8]."""
    W1 = _f32(W1)
    nh = W1.shape[1]
    if W1.shape != (8, nh, n_in):
        raise ValueError("W1 must be [8][n_hidden][26]")
    b1 = _f32(b1, (8, nh))
    W2 = _f32(W2, (8, 8, nh))
    b2 = _f32(b2, (8, 8))
    body = MAGIC + struct.pack("<7I", 2, n_in, nh, 8, int(activation), int(flags), 8)
    body += struct.pack("<2f", float(alpha), float(beta_scale))
    body += _f32(imin, (n_in,)).tobytes() + _f32(imax, (n_in,)).tobytes()
    for o in range(8):
        body += W1[o].tobytes() + b1[o].tobytes() + W2[o].tobytes() + b2[o].tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def write_paper_dir(path, W1, b1, W2, b2, imin, imax, omega, alpha=0.27, beta_scale=0.1,
                    n_in=26, activation=1, flags=1):
    """Version-3 artifact: W1 [K][nh][26], b1 [K][nh], W2 [K][8][nh], b2 [K][8],
    network k serving direction omega[k]."""
    W1 = _f32(W1)
    k, nh = W1.shape[0], W1.shape[1]
    if W1.shape != (k, nh, n_in):
        raise ValueError("W1 must be [K][n_hidden][26]")
    b1 = _f32(b1, (k, nh))
    W2 = _f32(W2, (k, 8, nh))
    b2 = _f32(b2, (k, 8))
    body = MAGIC + struct.pack("<7I", 3, n_in, nh, 8, int(activation), int(flags), k)
    body += struct.pack("<2f", float(alpha), float(beta_scale))
    body += _f32(imin, (n_in,)).tobytes() + _f32(imax, (n_in,)).tobytes()
    body += _f32(omega, (k, 3)).tobytes()
    for o in range(k):
        body += W1[o].tobytes() + b1[o].tobytes() + W2[o].tobytes() + b2[o].tobytes()
    with open(path, "wb") as f:
        f.write(body + struct.pack("<I", zlib.crc32(body) & 0xFFFFFFFF))


def read(path):
    data = open(path, "rb").read()
    if data[:8] != MAGIC:
        raise ValueError("not a DGSNANN1 artifact")
    version, nin, nh, nout, act, flags = struct.unpack("<6I", data[8:32])
    (crc,) = struct.unpack("<I", data[-4:])
    if crc != (zlib.crc32(data[:-4]) & 0xFFFFFFFF):
        raise ValueError("checksum mismatch")
    if version in (2, 3):
        (nnet,) = struct.unpack("<I", data[32:36])
        alpha, beta_scale = struct.unpack("<2f", data[36:44])
        f = np.frombuffer(data[44:-4], dtype="<f4")
        imin, imax = f[:nin].copy(), f[nin:2 * nin].copy()
        o = 2 * nin
        omega = None
        if version == 3:
            omega = f[o:o + 3 * nnet].reshape(nnet, 3).copy()
            o += 3 * nnet
        W1, b1, W2, b2 = [], [], [], []
        for _ in range(nnet):
            W1.append(f[o:o + nh * nin].reshape(nh, nin)); o += nh * nin
            b1.append(f[o:o + nh]); o += nh
            W2.append(f[o:o + nout * nh].reshape(nout, nh)); o += nout * nh
            b2.append(f[o:o + nout]); o += nout
        net = dict(W1=np.array(W1), b1=np.array(b1), W2=np.array(W2), b2=np.array(b2),
                   imin=imin, imax=imax, alpha=float(alpha), beta_scale=float(beta_scale),
                   act=int(act), flags=int(flags), version=int(version), kind="paper")
        if omega is not None:
            net["omega"] = omega
        return net
    f = np.frombuffer(data[32:-4], dtype="<f4")
    o = 0
    W1 = f[o:o + nh * nin].reshape(nh, nin); o += nh * nin
    b1 = f[o:o + nh]; o += nh
    W2 = f[o:o + nout * nh].reshape(nout, nh); o += nout * nh
    b2 = f[o:o + nout]
    return dict(W1=W1.copy(), b1=b1.copy(), W2=W2.copy(), b2=b2.copy(), act=int(act),
                flags=int(flags), version=int(version))

"""Writer/reader of the shallow-ANN artifact consumed by dgsn_ann_load.

Layout (little endian): b"DGSNANN1", u32 version=1, u32 n_in=24, u32 n_hidden,
u32 n_out=8, u32 activation (0 = ReLU, 1 = tanh), u32 flags, float32
W1[n_hidden][n_in], b1[n_hidden], W2[n_out][n_hidden], b2[n_out], u32 CRC-32
(IEEE) of all preceding bytes.
"""
import struct
import zlib

import numpy as np

MAGIC = b"DGSNANN1"


def write(path, W1, b1, W2, b2, activation=0, flags=0):
    W1 = np.ascontiguousarray(np.asarray(W1, np.float32))
    b1 = np.ascontiguousarray(np.asarray(b1, np.float32).reshape(-1))
    W2 = np.ascontiguousarray(np.asarray(W2, np.float32))
    b2 = np.ascontiguousarray(np.asarray(b2, np.float32).reshape(-1))
    nh, nin = W1.shape
    nout = W2.shape[0]
    if W2.shape != (nout, nh) or b1.shape != (nh,) or b2.shape != (nout,):
        raise ValueError("inconsistent ANN parameter shapes")
    body = MAGIC + struct.pack("<6I", 1, nin, nh, nout, int(activation), int(flags))
    body += W1.tobytes() + b1.tobytes() + W2.tobytes() + b2.tobytes()
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
    f = np.frombuffer(data[32:-4], dtype="<f4")
    o = 0
    W1 = f[o:o + nh * nin].reshape(nh, nin); o += nh * nin
    b1 = f[o:o + nh]; o += nh
    W2 = f[o:o + nout * nh].reshape(nout, nh); o += nout * nh
    b2 = f[o:o + nout]
    return dict(W1=W1.copy(), b1=b1.copy(), W2=W2.copy(), b2=b2.copy(), act=int(act),
                flags=int(flags), version=int(version))

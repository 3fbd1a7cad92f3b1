"""File format of the parameter-choice network's weights.

"GTMLP1\\0\\0", int32 inputs, hidden, outputs, nparams, then float32
params[nparams], fmin[inputs], fmax[inputs] (the feature range seen in
training; a graph outside it keeps the heuristic choice).
"""
import os
import struct

import numpy as np

MAGIC = b"GTMLP1\0\0"
INPUTS, HIDDEN, OUTPUTS = 16, 64, 32
NPARAMS = INPUTS * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN * OUTPUTS + OUTPUTS
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "gt_mlp.bin")


def save(path, params, fmin, fmax):
    params = np.asarray(params, dtype=np.float32).ravel()
    assert params.size == NPARAMS
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<4i", INPUTS, HIDDEN, OUTPUTS, NPARAMS))
        f.write(params.tobytes())
        f.write(np.asarray(fmin, dtype=np.float32).tobytes())
        f.write(np.asarray(fmax, dtype=np.float32).tobytes())


def load(path):
    with open(path, "rb") as f:
        data = f.read()
    if data[:8] != MAGIC:
        raise ValueError("not a GTMLP1 file")
    dims = struct.unpack("<4i", data[8:24])
    if dims != (INPUTS, HIDDEN, OUTPUTS, NPARAMS):
        raise ValueError(f"unexpected dimensions {dims}")
    arr = np.frombuffer(data[24:], dtype=np.float32)
    return arr[:NPARAMS].copy(), arr[NPARAMS:NPARAMS + INPUTS].copy(), arr[NPARAMS + INPUTS:].copy()

"""Seeded synthetic CSR inputs (R-MAT, uniform, geometric locality).

Shared by the oracle-side tests and the GPU side: this module only draws
inputs and holds none of the transposition's arithmetic (see gt_gen.c).
Arrays are numpy: offsets int64[n+1], indices int32[m], payload uint32[m]
(float32 bit patterns in [0, 1)) or None.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgtgen.so")
_SRC = os.path.join(_HERE, "gt_gen.c")

FAM_RMAT, FAM_UNIFORM, FAM_GEOMETRIC = 0, 1, 2
RMAT_G500 = (0.57, 0.19, 0.19, 0.05)


def build():
    """Compile the generator library in place (gcc + OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _SO, _SRC, "-lm"]
    subprocess.check_call(cmd)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_SO)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.gtgen_offsets.argtypes = [i32, i64, i32, i64, dbl, dbl, dbl, dbl, dbl, u64, i32, vp]
        lib.gtgen_offsets.restype = i32
        lib.gtgen_fill.argtypes = [i32, i64, i32, i64, dbl, dbl, dbl, dbl, dbl, u64, i32, vp, vp, vp]
        lib.gtgen_fill.restype = i32
        lib.gtgen_perm.argtypes = [u64, u64, i32, vp, vp, i64]
        lib.gtgen_perm.restype = i32
        lib.gtgen_draw.argtypes = [u64, u64, u64, u64]
        lib.gtgen_draw.restype = u64
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _scale_for(n):
    s = 0
    while (1 << s) < n:
        s += 1
    return s


def generate(family, n, ef, *, seed, permute=False, payload=False, probs=RMAT_G500, p_geom=0.01,
             scale=None):
    """Return (offsets, indices, payload-or-None) of a seeded synthetic CSR."""
    lib = _load()
    n = int(n)
    a, b, c, d = probs
    if scale is None:
        scale = _scale_for(n) if family == FAM_RMAT else 0
    O = np.empty(n + 1, dtype=np.int64)
    rc = lib.gtgen_offsets(family, n, scale, int(ef), a, b, c, d, p_geom, seed, int(permute), _ptr(O))
    if rc != 0:
        raise ValueError(f"gtgen_offsets failed ({rc})")
    m = int(O[-1])
    D = np.empty(m, dtype=np.int32)
    P = np.empty(m, dtype=np.uint32) if payload else None
    rc = lib.gtgen_fill(family, n, scale, int(ef), a, b, c, d, p_geom, seed, int(permute), _ptr(O), _ptr(D),
                        _ptr(P))
    if rc != 0:
        raise ValueError(f"gtgen_fill failed ({rc})")
    return O, D, P


def rmat(scale, ef, *, seed, permute=False, payload=False, probs=RMAT_G500, n=None):
    n = (1 << scale) if n is None else n
    return generate(FAM_RMAT, n, ef, seed=seed, permute=permute, payload=payload, probs=probs, scale=scale)


def uniform(n, ef, *, seed, permute=False, payload=False):
    return generate(FAM_UNIFORM, n, ef, seed=seed, permute=permute, payload=payload)


def geometric(n, ef, *, seed, p=0.01, permute=False, payload=False):
    return generate(FAM_GEOMETRIC, n, ef, seed=seed, permute=permute, payload=payload, p_geom=p)


def permutation(n, seed, ids, inverse=False):
    lib = _load()
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    out = np.empty_like(ids)
    rc = lib.gtgen_perm(n, seed, int(inverse), _ptr(ids), _ptr(out), ids.size)
    if rc != 0:
        raise ValueError("gtgen_perm failed")
    return out


def draw(seed, tag, ent, ctr):
    return int(_load().gtgen_draw(seed, tag, ent, ctr))


# ---------------------------------------------------------------------------
# Named workloads.  Seeds: the tiny R-MAT uses seed 1; the others use 2, 3, 4,
# 26 and 5 (batch) so that every workload is reproducible from its name.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "rmat16": dict(kind="rmat", scale=16, ef=16, seed=1, permute=False, payload=False),
    "rmat24p": dict(kind="rmat", scale=24, ef=16, seed=2, permute=True, payload=True),
    "uniform26": dict(kind="uniform", n=1 << 26, ef=16, seed=3, payload=False),
    "geom26": dict(kind="geometric", n=1 << 26, ef=16, seed=3, p=0.01, payload=False),
    "rmat26": dict(kind="rmat", scale=26, ef=16, seed=26, permute=False, payload=False),
    "rmat26p": dict(kind="rmat", scale=26, ef=16, seed=26, permute=True, payload=False),
    "rmat28p": dict(kind="rmat", scale=28, ef=16, seed=4, permute=True, payload=False),
}


def workload(name):
    w = WORKLOADS[name]
    if w["kind"] == "rmat":
        return rmat(w["scale"], w["ef"], seed=w["seed"], permute=w["permute"], payload=w["payload"])
    if w["kind"] == "uniform":
        return uniform(w["n"], w["ef"], seed=w["seed"], payload=w["payload"])
    return geometric(w["n"], w["ef"], seed=w["seed"], p=w["p"], payload=w["payload"])


def batch_specs(count=512, seed=5):
    """Per-graph specs of the uneven batch: n = floor(2^x), x ~ U[10, 22];
    ef in {4, 8, 16, 32}; family uniform over {R-MAT, uniform, geometric};
    R-MAT a ~ U[.45, .65], b = c = (1 - a - .05)/2, d = .05, permuted with
    probability 1/2; geometric p log-uniform in [1e-3, 1e-1]; a payload on
    exactly half of the graphs (chosen by a seeded shuffle)."""
    rs = []
    u = lambda i, k: (draw(seed, 7, i, k) >> 11) * (1.0 / 9007199254740992.0)
    order = sorted(range(count), key=lambda i: draw(seed, 8, i, 0))
    with_payload = set(order[: count // 2])
    for i in range(count):
        x = 10.0 + 12.0 * u(i, 0)
        n = int(2.0 ** x)
        ef = (4, 8, 16, 32)[draw(seed, 7, i, 1) % 4]
        fam = draw(seed, 7, i, 2) % 3
        spec = dict(n=n, ef=ef, family=fam, seed=1000000 + 7919 * i + seed, payload=(i in with_payload))
        if fam == FAM_RMAT:
            a = 0.45 + 0.20 * u(i, 3)
            bc = (1.0 - a - 0.05) / 2
            spec.update(probs=(a, bc, bc, 0.05), permute=bool(draw(seed, 7, i, 4) & 1))
        elif fam == FAM_GEOMETRIC:
            spec.update(p_geom=10.0 ** (-3.0 + 2.0 * u(i, 5)))
        rs.append(spec)
    return rs


def from_spec(spec):
    return generate(spec["family"], spec["n"], spec["ef"], seed=spec["seed"], permute=spec.get("permute", False),
                    payload=spec["payload"], probs=spec.get("probs", RMAT_G500), p_geom=spec.get("p_geom", 0.01))
